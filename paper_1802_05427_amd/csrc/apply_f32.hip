// Block filtering Hhat[O_b] = W_b H_LS[I_b] (eq. 12 per block of Sec. IV-B)
// on the FP32 matrix cores of gfx950.
//
// The complex product is done as a real GEMM with the 2B x 2Wn real embedding
// of W (see internal.h), which keeps the data in its interleaved (re, im)
// layout: window rows j, j+1 of a column are 4 consecutive floats and so are
// 2 consecutive outputs.  v_mfma_f32_16x16x4f32 is used with a permuted
// contraction order: within a group of 16 reals (8 complex window rows), lane
// (i16, q) holds reals 4q..4q+3 of its row / column in one float4 and feeds
// element i of it to k-step i, for both operands.  The product is unchanged
// (the contraction order is only permuted), and every operand load is a
// 16-byte vector load.
//
// One wave (64 lanes) = one workgroup computes, for one block b and one row
// group, RT 16-row tiles x CT 16-column tiles.  Filters ("A") are read from
// the pre-laid-out bank in L2; H_LS columns ("B") come straight from HBM
// (unfused) or from LDS after an in-register despread of the pilot symbols
// (fused: the wave first reads y[s, m, 0..K-1, window chunk] for the antennas
// of its 16*CT columns, undoes the cover code with a K-point DFT, multiplies
// by conj(x_k[n]) / K and stages the LS values in LDS).  The block index runs
// fastest over consecutive tiles and tiles are remapped so that each XCD
// processes a contiguous range: neighbouring (overlapping) windows of a column
// tile are read by the same L2.
#include "dft.h"
#include "internal.h"

namespace lmmse {

typedef float floatx4 __attribute__((ext_vector_type(4)));

struct ApplyArgs {
    const float4* wbank;
    const int* starts;
    const int* classes;
    const float2* x;       // H_LS [cols][N] (unfused) or y [S*M][K][N] (fused)
    const float2* pilots;  // [K][N] (fused only)
    float2* out;           // [cols][N]
    long long ncols;       // S*M*K
    long long n_tiles;
    int N, B, Wn, G8, Rpad, nb, rgroups;
    int vec_store;         // N, B even and out 16-byte aligned: float4 stores
    float invK;
};

__device__ __forceinline__ long long xcd_remap(long long id, long long total) {
    const long long NX = 8;
    const long long q = total / NX, r = total % NX;
    const long long x = id % NX, k = id / NX;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ __forceinline__ float f4c(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

template <int RT, int CT>
__device__ __forceinline__ void mfma_group(floatx4 (&acc)[RT][CT], const float4 (&av)[RT],
                                           const float4 (&xv)[CT]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(f4c(av[rt], i), f4c(xv[ct], i),
                                                                   acc[rt][ct], 0, 0, 0);
}

template <int RT, int CT>
__device__ __forceinline__ void store_tiles(const ApplyArgs& a, const floatx4 (&acc)[RT][CT],
                                            long long c0, int b, int rg, int l16, int q) {
    const bool vec = a.vec_store != 0;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const long long col = c0 + ct * 16 + l16;
        if (col >= a.ncols) continue;
        float2* op = a.out + col * a.N + (long long)b * a.B;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int o = (((rg * RT + rt) * 16) + 4 * q) >> 1;
            const floatx4 v = acc[rt][ct];
            if (o + 1 < a.B) {
                if (vec) {
                    *reinterpret_cast<float4*>(op + o) = make_float4(v[0], v[1], v[2], v[3]);
                } else {
                    op[o] = make_float2(v[0], v[1]);
                    op[o + 1] = make_float2(v[2], v[3]);
                }
            } else if (o < a.B) {
                op[o] = make_float2(v[0], v[1]);
            }
        }
    }
}

template <int RT, int CT>
__global__ __launch_bounds__(64) void apply_f32_kernel(ApplyArgs a) {
    const int lane = threadIdx.x, l16 = lane & 15, q = lane >> 4;
    long long t = xcd_remap(blockIdx.x, a.n_tiles);
    const int rg = (int)(t % a.rgroups);
    t /= a.rgroups;
    const int b = (int)(t % a.nb);
    const long long c0 = (t / a.nb) * (16 * CT);
    const int s0 = a.starts[b], cls = a.classes[b];

    floatx4 acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};

    const float4* wp = a.wbank + ((size_t)cls * a.G8 * a.Rpad + (size_t)rg * RT * 16 + l16) * 4 + q;
    const float2* xp[CT];
    bool cv[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const long long col = c0 + ct * 16 + l16;
        cv[ct] = col < a.ncols;
        xp[ct] = a.x + (cv[ct] ? col : 0) * a.N + s0;
    }
    for (int g = 0; g < a.G8; ++g) {
        float4 av[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) av[rt] = wp[((size_t)g * a.Rpad + rt * 16) * 4];
        float4 xv[CT];
        const int j = 8 * g + 2 * q;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            float2 u0 = make_float2(0.f, 0.f), u1 = make_float2(0.f, 0.f);
            if (cv[ct] && j < a.Wn) u0 = xp[ct][j];
            if (cv[ct] && j + 1 < a.Wn) u1 = xp[ct][j + 1];
            xv[ct] = make_float4(u0.x, u0.y, u1.x, u1.y);
        }
        mfma_group<RT, CT>(acc, av, xv);
    }
    store_tiles<RT, CT>(a, acc, c0, b, rg, l16, q);
}

template <int RT, int CT, int KF>
__global__ __launch_bounds__(64) void apply_f32_fused_kernel(ApplyArgs a) {
    static_assert((16 * CT) % KF == 0, "tile must hold whole antennas");
    constexpr int NA = 16 * CT / KF;   // antennas per tile
    constexpr int XS = 18;             // LDS column stride in complex (16 rows + pad)
    __shared__ float4 xs4[16 * CT * XS / 2];
    float2* xs2 = reinterpret_cast<float2*>(xs4);

    const int lane = threadIdx.x, l16 = lane & 15, q = lane >> 4;
    long long t = xcd_remap(blockIdx.x, a.n_tiles);
    const int rg = (int)(t % a.rgroups);
    t /= a.rgroups;
    const int b = (int)(t % a.nb);
    const long long c0 = (t / a.nb) * (16 * CT);
    const int s0 = a.starts[b], cls = a.classes[b];
    const long long ant0 = c0 / KF, n_ant = a.ncols / KF;

    floatx4 acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};

    const float4* wp = a.wbank + ((size_t)cls * a.G8 * a.Rpad + (size_t)rg * RT * 16 + l16) * 4 + q;
    const int nchunks = (a.Wn + 15) >> 4;
    for (int cc = 0; cc < nchunks; ++cc) {
        // despread 16 window rows of every antenna of the tile into LDS
        for (int pi = lane; pi < NA * 16; pi += 64) {
            const int aa = pi >> 4, r = pi & 15;
            const int j = cc * 16 + r;
            const long long ant = ant0 + aa;
            float2* dst = xs2 + aa * KF * XS + r;
            if (j < a.Wn && ant < n_ant) {
                const int n = s0 + j;
                const float2* yp = a.x + ant * KF * (long long)a.N + n;
                float2 v[KF], z[KF];
#pragma unroll
                for (int tt = 0; tt < KF; ++tt) v[tt] = yp[(long long)tt * a.N];
                Dft<KF>::run(v, z, nullptr);
#pragma unroll
                for (int k = 0; k < KF; ++k) {
                    const float2 h = cmulc(z[k], a.pilots[(long long)k * a.N + n]);
                    dst[k * XS] = make_float2(h.x * a.invK, h.y * a.invK);
                }
            } else {
#pragma unroll
                for (int k = 0; k < KF; ++k) dst[k * XS] = make_float2(0.f, 0.f);
            }
        }
        __syncthreads();
#pragma unroll
        for (int gg = 0; gg < 2; ++gg) {
            const int g = 2 * cc + gg;
            if (g < a.G8) {
                float4 av[RT];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) av[rt] = wp[((size_t)g * a.Rpad + rt * 16) * 4];
                float4 xv[CT];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) xv[ct] = xs4[(ct * 16 + l16) * (XS / 2) + 4 * gg + q];
                mfma_group<RT, CT>(acc, av, xv);
            }
        }
        __syncthreads();
    }
    store_tiles<RT, CT>(a, acc, c0, b, rg, l16, q);
}

static constexpr int kCT = 3;

bool apply_fusable(const Plan& p) {
    const int K = p.d.K;
    return K == 1 || K == 2 || K == 4 || K == 12 || K == 24;
}

hipError_t launch_apply_f32(const Plan& p, int slots, const float2* x, const float2* pilots,
                            bool fused, float2* out, hipStream_t st) {
    ApplyArgs a;
    a.wbank = p.wf32;
    a.starts = p.d_starts;
    a.classes = p.d_classes;
    a.x = x;
    a.pilots = pilots;
    a.out = out;
    a.ncols = (long long)slots * p.d.M * p.d.K;
    a.N = p.d.N;
    a.B = p.d.B;
    a.Wn = p.d.Wn;
    a.G8 = p.G8;
    a.Rpad = p.Rpad;
    a.nb = p.nb;
    a.rgroups = p.rgroups;
    a.invK = 1.0f / (float)p.d.K;
    a.vec_store = (((a.N | a.B) & 1) == 0 && ((uintptr_t)out & 15) == 0) ? 1 : 0;
    const long long ctiles = (a.ncols + 16 * kCT - 1) / (16 * kCT);
    a.n_tiles = ctiles * p.nb * p.rgroups;
    if (a.n_tiles == 0) return hipSuccess;
    const dim3 grid((unsigned)a.n_tiles), block(64);
    if (!fused) {
        switch (p.RT) {
#define LMMSE_AF(R)                                                                     \
    case R:                                                                             \
        hipLaunchKernelGGL((apply_f32_kernel<R, kCT>), grid, block, 0, st, a);           \
        break;
            LMMSE_AF(1) LMMSE_AF(2) LMMSE_AF(4) LMMSE_AF(8) LMMSE_AF(9) LMMSE_AF(13)
            LMMSE_AF(15) LMMSE_AF(17)
#undef LMMSE_AF
            default:
                return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
#define LMMSE_AFF(R, KK)                                                                \
    case R:                                                                             \
        hipLaunchKernelGGL((apply_f32_fused_kernel<R, kCT, KK>), grid, block, 0, st, a); \
        break;
#define LMMSE_AFK(KK)                                                                    \
    case KK:                                                                             \
        switch (p.RT) {                                                                  \
            LMMSE_AFF(1, KK) LMMSE_AFF(2, KK) LMMSE_AFF(4, KK) LMMSE_AFF(8, KK)          \
            LMMSE_AFF(9, KK) LMMSE_AFF(13, KK) LMMSE_AFF(15, KK) LMMSE_AFF(17, KK)       \
            default: return hipErrorInvalidValue;                                        \
        }                                                                                \
        break;
    switch (p.d.K) {
        LMMSE_AFK(1) LMMSE_AFK(2) LMMSE_AFK(4) LMMSE_AFK(12) LMMSE_AFK(24)
        default:
            return hipErrorInvalidValue;
    }
#undef LMMSE_AFK
#undef LMMSE_AFF
    return hipGetLastError();
}

}  // namespace lmmse
