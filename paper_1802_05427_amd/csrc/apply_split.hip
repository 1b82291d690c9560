// Block filtering (eq. 12 per block of Sec. IV-B) with split-precision
// products on the BF16 / FP16 matrix cores of gfx950.
//
// Every FP32 operand x is split as x = hi + lo with hi = round(x) and
// lo = round(x - hi) in the 16-bit format (round to nearest even), and the
// product W X is formed as hi_W hi_X + lo_W hi_X + hi_W lo_X with FP32
// accumulation (lo_W lo_X is dropped).  BF16 has the FP32 exponent range, so
// its parts are used as they are.  FP16 lo parts are scaled by 2^11 to stay
// clear of the subnormal range, and the hi_W hi_X product uses the exactly
// representable 2^11 hi_W, so the accumulator holds 2^11 W X and one scale by
// 2^-11 at the store undoes it.  FP16 assumes |W| < 32 and |h_ls| < 65504.
//
// The structure follows the FP32 kernel (apply_f32.hip): 4 waves x 3 column
// tiles = 192 columns per workgroup, RT <= 13 16-row tiles of the real
// embedding, the window streamed in chunks of 16 complex rows (32 reals = the
// K of one v_mfma_f32_16x16x32_{bf16,f16}), the next chunk's raw inputs
// loaded into registers before the current chunk's MFMAs.  Lane (i16, kq) of
// an operand holds reals 8kq..8kq+7 of its row / column (one 16-byte LDS
// read).  The LS chunk is split once, when it is written to LDS.
#include "dft.h"
#include "internal.h"

namespace lmmse {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

struct SplitArgs {
    const uint4* p0;       // A part multiplying hi_X: BF16 hi_W, FP16 2^11 hi_W
    const uint4* p1;       // A part multiplying lo_X: hi_W
    const uint4* p2;       // A part multiplying hi_X: BF16 lo_W, FP16 2^11 lo_W
    const int* starts;
    const int* classes;
    const float2* x;
    const float2* pilots;
    float2* out;
    long long ncols;
    long long n_tiles;
    int N, B, Wn, G16, Rpad, nb, rgroups;
    int vec_store;
    float invK;
    float out_scale;
};

__device__ __forceinline__ long long xcd_remap_s(long long id, long long total) {
    const long long NX = 8;
    const long long q = total / NX, r = total % NX;
    const long long x = id % NX, k = id / NX;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <bool FP16>
__device__ __forceinline__ void split2(float v, uint16_t& h, uint16_t& l) {
    if constexpr (FP16) {
        const _Float16 hh = (_Float16)v;
        const _Float16 ll = (_Float16)((v - (float)hh) * 2048.0f);
        h = __builtin_bit_cast(uint16_t, hh);
        l = __builtin_bit_cast(uint16_t, ll);
    } else {
        const __bf16 hh = (__bf16)v;
        const __bf16 ll = (__bf16)(v - (float)hh);
        h = __builtin_bit_cast(uint16_t, hh);
        l = __builtin_bit_cast(uint16_t, ll);
    }
}

// hi and lo of one complex value, each as a packed (re, im) pair
template <bool FP16>
__device__ __forceinline__ void split_c(float2 v, uint32_t& hi, uint32_t& lo) {
    uint16_t hr, lr, hi_, li;
    split2<FP16>(v.x, hr, lr);
    split2<FP16>(v.y, hi_, li);
    hi = (uint32_t)hr | ((uint32_t)hi_ << 16);
    lo = (uint32_t)lr | ((uint32_t)li << 16);
}

template <bool FP16>
__device__ __forceinline__ floatx4 mma(const uint4& a, const uint4& b, floatx4 c) {
    if constexpr (FP16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

constexpr int sCT = 3;                     // column tiles per wave
constexpr int sThreads = 256;              // 4 waves
constexpr int sCols = 16 * sCT * 4;        // 192
constexpr int sXS = 20;                    // LDS column stride in uint32 (16 rows + pad)

template <int KF>
struct SRaw {
    static constexpr int NPAIR = KF == 0 ? sCols * 16 : (sCols / KF) * 16;
    static constexpr int TX = (NPAIR + sThreads - 1) / sThreads;
    static constexpr int KV = KF == 0 ? 1 : KF;
    float2 v[TX][KV];
};

template <int KF>
__device__ __forceinline__ void split_load_raw(const SplitArgs& a, int tid, int cc, int s0,
                                               long long c0, SRaw<KF>& R) {
    using CR = SRaw<KF>;
#pragma unroll
    for (int u = 0; u < CR::TX; ++u) {
        const int i = tid + u * sThreads;
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

// LS values of chunk cc, split into hi / lo parts, into LDS.
template <int KF, bool FP16>
__device__ __forceinline__ void split_store_ls(const SplitArgs& a, int tid, int cc, int s0,
                                               const SRaw<KF>& R, uint32_t* xh, uint32_t* xl) {
    using CR = SRaw<KF>;
#pragma unroll
    for (int u = 0; u < CR::TX; ++u) {
        const int i = tid + u * sThreads;
        if (i >= CR::NPAIR) continue;
        const int cq = i >> 4, r = i & 15;
        if constexpr (KF == 0) {
            uint32_t h, l;
            split_c<FP16>(R.v[u][0], h, l);
            xh[cq * sXS + r] = h;
            xl[cq * sXS + r] = l;
        } else {
            const int j = cc * 16 + r;
            const bool live = j < a.Wn;
            const int n = live ? s0 + j : 0;
            const int cb = cq * KF * sXS + r;
            float2 z[KF];
            Dft<KF>::run(R.v[u], z, nullptr);
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                float2 h = cmulc(z[k], a.pilots[(long long)k * a.N + n]);
                h = live ? make_float2(h.x * a.invK, h.y * a.invK) : make_float2(0.f, 0.f);
                uint32_t hh, ll;
                split_c<FP16>(h, hh, ll);
                xh[cb + k * sXS] = hh;
                xl[cb + k * sXS] = ll;
            }
        }
    }
}

template <int RT, int KF>
constexpr int split_min_blocks() { return (KF == 24 || (RT >= 13 && KF <= 2)) ? 1 : 2; }

// 4 waves x 3 column tiles, RT <= 13 row tiles; per chunk of 16 window rows:
// filter parts and split LS values into LDS, barrier, MFMAs, barrier; the
// raw inputs of the next chunk are loaded into registers before the MFMAs.
template <int RT, int KF, bool FP16>
__global__ __launch_bounds__(sThreads, (split_min_blocks<RT, KF>())) void apply_split_kernel(SplitArgs a) {
    __shared__ uint4 xh4[sCols * sXS / 4];
    __shared__ uint4 xl4[sCols * sXS / 4];
    __shared__ uint4 w4[3 * RT * 64];          // [part][kq][row]
    uint32_t* xh = reinterpret_cast<uint32_t*>(xh4);
    uint32_t* xl = reinterpret_cast<uint32_t*>(xl4);

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l16 = lane & 15, kq = lane >> 4;
    long long t = xcd_remap_s(blockIdx.x, a.n_tiles);
    const int rg = (int)(t % a.rgroups);
    t /= a.rgroups;
    const int b = (int)(t % a.nb);
    const long long c0 = (t / a.nb) * sCols;
    const int s0 = a.starts[b], cls = a.classes[b];
    const size_t wbase = ((size_t)cls * a.G16 * a.Rpad + (size_t)rg * RT * 16) * 4;
    const int nchunks = a.G16;

    floatx4 acc[RT][sCT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < sCT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};

    SRaw<KF> raw;
    split_load_raw<KF>(a, tid, 0, s0, c0, raw);
    for (int cc = 0; cc < nchunks; ++cc) {
        const size_t wofs = wbase + (size_t)cc * a.Rpad * 4;
        // q-major LDS copy ([part][kq][row]): conflict-free 16-byte reads
        for (int i = tid; i < RT * 64; i += sThreads) {
            const int li = (i & 3) * RT * 16 + (i >> 2);
            w4[li] = a.p0[wofs + i];
            w4[RT * 64 + li] = a.p1[wofs + i];
            w4[2 * RT * 64 + li] = a.p2[wofs + i];
        }
        split_store_ls<KF, FP16>(a, tid, cc, s0, raw, xh, xl);
        if (cc + 1 < nchunks) split_load_raw<KF>(a, tid, cc + 1, s0, c0, raw);
        __syncthreads();
        uint4 bh[sCT], bl[sCT];
#pragma unroll
        for (int ct = 0; ct < sCT; ++ct) {
            const int c = (wave * sCT + ct) * 16 + l16;
            bh[ct] = xh4[c * (sXS / 4) + kq];
            bl[ct] = xl4[c * (sXS / 4) + kq];
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int wi = kq * RT * 16 + rt * 16 + l16;
            const uint4 a0 = w4[wi], a1 = w4[RT * 64 + wi], a2 = w4[2 * RT * 64 + wi];
            // three independent column tiles between dependent products
#pragma unroll
            for (int ct = 0; ct < sCT; ++ct) acc[rt][ct] = mma<FP16>(a0, bh[ct], acc[rt][ct]);
#pragma unroll
            for (int ct = 0; ct < sCT; ++ct) acc[rt][ct] = mma<FP16>(a2, bh[ct], acc[rt][ct]);
#pragma unroll
            for (int ct = 0; ct < sCT; ++ct) acc[rt][ct] = mma<FP16>(a1, bl[ct], acc[rt][ct]);
        }
        __syncthreads();
    }

    const bool vec = a.vec_store != 0;
    const float sc = a.out_scale;
#pragma unroll
    for (int ct = 0; ct < sCT; ++ct) {
        const long long col = c0 + (wave * sCT + ct) * 16 + l16;
        if (col >= a.ncols) continue;
        float2* op = a.out + col * a.N + (long long)b * a.B;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int o = (((rg * RT + rt) * 16) + 4 * kq) >> 1;
            const floatx4 v = acc[rt][ct];
            if (o + 1 < a.B) {
                if (vec) {
                    *reinterpret_cast<float4*>(op + o) =
                        make_float4(v[0] * sc, v[1] * sc, v[2] * sc, v[3] * sc);
                } else {
                    op[o] = make_float2(v[0] * sc, v[1] * sc);
                    op[o + 1] = make_float2(v[2] * sc, v[3] * sc);
                }
            } else if (o < a.B) {
                op[o] = make_float2(v[0] * sc, v[1] * sc);
            }
        }
    }
}

template <bool FP16>
static hipError_t launch_split_t(const SplitArgs& a, int RT, int kf, hipStream_t st) {
    const dim3 grid((unsigned)a.n_tiles), block(sThreads);
#define LMMSE_AS(R, KK)                                                                  \
    case R:                                                                              \
        hipLaunchKernelGGL((apply_split_kernel<R, KK, FP16>), grid, block, 0, st, a);    \
        break;
#define LMMSE_ASK(KK)                                                                    \
    case KK:                                                                             \
        switch (RT) {                                                                    \
            LMMSE_AS(1, KK) LMMSE_AS(2, KK) LMMSE_AS(4, KK) LMMSE_AS(8, KK)              \
            LMMSE_AS(9, KK) LMMSE_AS(13, KK)                                             \
            default: return hipErrorInvalidValue;                                        \
        }                                                                                \
        break;
    switch (kf) {
        LMMSE_ASK(0) LMMSE_ASK(1) LMMSE_ASK(2) LMMSE_ASK(4) LMMSE_ASK(12) LMMSE_ASK(24)
        default:
            return hipErrorInvalidValue;
    }
#undef LMMSE_ASK
#undef LMMSE_AS
    return hipGetLastError();
}

hipError_t launch_apply_split(const Plan& p, int slots, const float2* x, const float2* pilots,
                              bool fused, float2* out, hipStream_t st) {
    const bool fp16 = p.d.precision == LMMSE_FP16X3;
    SplitArgs a;
    a.p0 = reinterpret_cast<const uint4*>(fp16 ? p.whs : p.whi);
    a.p1 = reinterpret_cast<const uint4*>(p.whi);
    a.p2 = reinterpret_cast<const uint4*>(p.wlo);
    a.starts = p.d_starts;
    a.classes = p.d_classes;
    a.x = x;
    a.pilots = pilots;
    a.out = out;
    a.ncols = (long long)slots * p.d.M * p.d.K;
    a.N = p.d.N;
    a.B = p.d.B;
    a.Wn = p.d.Wn;
    a.G16 = p.G16;
    a.Rpad = p.Rpad;
    a.nb = p.nb;
    a.rgroups = p.rgroups;
    a.invK = 1.0f / (float)p.d.K;
    a.out_scale = fp16 ? 1.0f / 2048.0f : 1.0f;
    a.vec_store = (((a.N | a.B) & 1) == 0 && ((uintptr_t)out & 15) == 0) ? 1 : 0;
    const long long ctiles = (a.ncols + sCols - 1) / sCols;
    a.n_tiles = ctiles * p.nb * p.rgroups;
    if (a.n_tiles == 0) return hipSuccess;
    const int kf = fused ? p.d.K : 0;
    return fp16 ? launch_split_t<true>(a, p.RT, kf, st) : launch_split_t<false>(a, p.RT, kf, st);
}

}  // namespace lmmse
