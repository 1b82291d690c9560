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
// (only the contraction order is permuted) and every operand read is a
// 16-byte LDS read.
//
// A workgroup (4 waves) computes one block b, one row group (RT 16-row tiles)
// and 192 columns; wave w owns columns [48w, 48w+48) (3 column tiles).  The
// window is streamed in chunks of 16 complex rows: the workgroup copies the
// chunk's filter rows (shared by all 4 waves) and its LS values into LDS, then
// every wave runs RT x 3 x 8 MFMAs.  The raw inputs of chunk c+1 are loaded
// into registers before the MFMAs of chunk c, and two workgroups share a CU,
// so memory latency overlaps the matrix work.  LS values come from
// H_LS (unfused) or are made on the fly from the pilot symbols (fused: one
// thread per (antenna, subcarrier) reads y[s,m,0..K-1,n], undoes the cover
// code with a K-point DFT and multiplies by conj(x_k[n]) / K).  The block index
// runs fastest over consecutive tiles and tiles are remapped so that each XCD
// takes a contiguous range: the overlapping windows of neighbouring blocks of
// a column group are read through the same L2.
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

constexpr int kCT = 3;                 // column tiles per wave
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kCols = 16 * kCT * kWaves;   // 192 columns per workgroup
constexpr int kXS = 18;                // LDS column stride in complex (16 rows + pad)

// Raw LS-path inputs one thread holds for one chunk (window rows [16cc, 16cc+16)).
template <int KF>
struct RawRegs {
    static constexpr int NPAIR = KF == 0 ? kCols * 16 : (kCols / KF) * 16;
    static constexpr int TX = (NPAIR + kThreads - 1) / kThreads;
    static constexpr int KV = KF == 0 ? 1 : KF;
    float2 v[TX][KV];
};

template <int KF>
__device__ __forceinline__ void load_raw(const ApplyArgs& a, int tid, int cc, int s0, long long c0,
                                         RawRegs<KF>& R) {
    using CR = RawRegs<KF>;
#pragma unroll
    for (int u = 0; u < CR::TX; ++u) {
        const int i = tid + u * kThreads;
        const int cq = i >> 4, r = i & 15;
        const int j = cc * 16 + r;
        if constexpr (KF == 0) {
            const long long col = c0 + cq;
            R.v[u][0] = (i < CR::NPAIR && j < a.Wn && col < a.ncols) ? a.x[col * a.N + s0 + j]
                                                                    : make_float2(0.f, 0.f);
        } else {
            const long long ant = c0 / KF + cq;
            const bool live = i < CR::NPAIR && j < a.Wn && ant < a.ncols / KF;
            const float2* yp = a.x + ant * KF * (long long)a.N + s0 + j;
#pragma unroll
            for (int tt = 0; tt < KF; ++tt)
                R.v[u][tt] = live ? yp[(long long)tt * a.N] : make_float2(0.f, 0.f);
        }
    }
}

// LS values of chunk cc into LDS: straight (unfused) or despread (fused).
template <int KF>
__device__ __forceinline__ void store_ls(const ApplyArgs& a, int tid, int cc, int s0,
                                         const RawRegs<KF>& R, float2* xs2) {
    using CR = RawRegs<KF>;
#pragma unroll
    for (int u = 0; u < CR::TX; ++u) {
        const int i = tid + u * kThreads;
        if (i >= CR::NPAIR) continue;
        const int cq = i >> 4, r = i & 15;
        if constexpr (KF == 0) {
            xs2[cq * kXS + r] = R.v[u][0];
        } else {
            const int j = cc * 16 + r;
            const bool live = j < a.Wn;
            const int n = live ? s0 + j : 0;
            float2* dst = xs2 + cq * KF * kXS + r;
            float2 z[KF];
            Dft<KF>::run(R.v[u], z, nullptr);
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                const float2 h = cmulc(z[k], a.pilots[(long long)k * a.N + n]);
                dst[k * kXS] = live ? make_float2(h.x * a.invK, h.y * a.invK) : make_float2(0.f, 0.f);
            }
        }
    }
}

// RT row tiles x 3 column tiles per wave, 4 waves, 2 workgroups per CU.  Per
// chunk: filter rows and LS values into LDS, barrier, MFMAs, barrier; the
// raw inputs of the next chunk are loaded into registers before the MFMAs so
// that their memory latency is hidden behind them.
// Two workgroups per CU where the registers allow it (tall row groups and
// K = 24 run one per CU rather than spill).
template <int RT, int KF>
constexpr int min_blocks() { return (RT <= 13 && KF != 24) ? 2 : 1; }

template <int RT, int KF>
__global__ __launch_bounds__(kThreads, (min_blocks<RT, KF>())) void apply_f32_kernel(ApplyArgs a) {
    __shared__ float4 xs4[kCols * kXS / 2];   // LS chunk: [col][16 rows]
    __shared__ float4 ws4[2 * RT * 64];       // filter chunk: [g][q][row]
    float2* xs2 = reinterpret_cast<float2*>(xs4);

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l16 = lane & 15, q = lane >> 4;
    long long t = xcd_remap(blockIdx.x, a.n_tiles);
    const int rg = (int)(t % a.rgroups);
    t /= a.rgroups;
    const int b = (int)(t % a.nb);
    const long long c0 = (t / a.nb) * kCols;
    const int s0 = a.starts[b], cls = a.classes[b];
    const float4* wsrc = a.wbank + ((size_t)cls * a.G8 * a.Rpad + (size_t)rg * RT * 16) * 4;
    const int nchunks = (a.Wn + 15) >> 4;

    floatx4 acc[RT][kCT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < kCT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};

    RawRegs<KF> raw;
    load_raw<KF>(a, tid, 0, s0, c0, raw);
    for (int cc = 0; cc < nchunks; ++cc) {
        // LDS copy is q-major ([g][q][row]) so that the 16 rows a lane group
        // reads are consecutive 16-byte words (no bank conflicts)
        for (int i = tid; i < 2 * RT * 64; i += kThreads) {
            const int gg = i / (RT * 64), rem = i - gg * (RT * 64);
            const int g = 2 * cc + gg;
            const int row = rem >> 2, qq = rem & 3;
            ws4[gg * RT * 64 + qq * RT * 16 + row] =
                g < a.G8 ? wsrc[(size_t)g * a.Rpad * 4 + rem] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        store_ls<KF>(a, tid, cc, s0, raw, xs2);
        if (cc + 1 < nchunks) load_raw<KF>(a, tid, cc + 1, s0, c0, raw);
        __syncthreads();
#pragma unroll
        for (int gg = 0; gg < 2; ++gg) {
            float4 xv[kCT];
#pragma unroll
            for (int ct = 0; ct < kCT; ++ct)
                xv[ct] = xs4[((wave * kCT + ct) * 16 + l16) * (kXS / 2) + 4 * gg + q];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const float4 av = ws4[gg * RT * 64 + q * RT * 16 + rt * 16 + l16];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int ct = 0; ct < kCT; ++ct)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            f4c(av, i), f4c(xv[ct], i), acc[rt][ct], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // lane (l16, q) of tile (rt, ct) holds real rows 16rt + 4q .. +3 of its
    // column: complex outputs o, o+1 of the block
    const bool vec = a.vec_store != 0;
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) {
        const long long col = c0 + (wave * kCT + ct) * 16 + l16;
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
    const long long ctiles = (a.ncols + kCols - 1) / kCols;
    a.n_tiles = ctiles * p.nb * p.rgroups;
    if (a.n_tiles == 0) return hipSuccess;
    const dim3 grid((unsigned)a.n_tiles);
    const int kf = fused ? p.d.K : 0;
#define LMMSE_AF(R, KK)                                                                  \
    case R:                                                                              \
        hipLaunchKernelGGL((apply_f32_kernel<R, KK>), grid, dim3(kThreads), 0, st, a);   \
        break;
#define LMMSE_AFK(KK)                                                                    \
    case KK:                                                                             \
        switch (p.RT) {                                                                  \
            LMMSE_AF(1, KK) LMMSE_AF(2, KK) LMMSE_AF(4, KK) LMMSE_AF(8, KK)              \
            LMMSE_AF(9, KK) LMMSE_AF(13, KK) LMMSE_AF(15, KK) LMMSE_AF(17, KK)           \
            default: return hipErrorInvalidValue;                                        \
        }                                                                                \
        break;
    switch (kf) {
        LMMSE_AFK(0) LMMSE_AFK(1) LMMSE_AFK(2) LMMSE_AFK(4) LMMSE_AFK(12) LMMSE_AFK(24)
        default:
            return hipErrorInvalidValue;
    }
#undef LMMSE_AFK
#undef LMMSE_AF
    return hipGetLastError();
}

}  // namespace lmmse
