// Block filtering (eq. 12 per block of Sec. IV-B) with split-precision
// products on the BF16 / FP16 matrix cores of gfx950.
//
// Every FP32 operand x is split as x = hi + lo with hi = round(x) and
// lo = round(x - hi) in the 16-bit format (round to nearest even), and the
// product W X is formed as hi_W hi_X + lo_W hi_X + hi_W lo_X with FP32
// accumulation (lo_W lo_X is dropped).  BF16 has the FP32 exponent range, so
// its parts are used as they are.  FP16 lo parts are scaled by 2^11 to stay
// clear of the subnormal range, and the hi_W hi_X product uses 2^11 hi_W
// (exact: a power-of-two scaling, formed in registers from hi_W), so the
// accumulator holds 2^11 W X and one scale by 2^-11 at the store undoes it.
// FP16 needs |W| < 32 (checked when the bank is packed) and |s h_ls| < 65504
// for the plan's power-of-two input scale s (the LS values are multiplied by
// s before the split and the output by 1/s, both exact); a value past that
// records LMMSE_ERR_RANGE in the plan's status word.  Below about 1.2e-4 the
// FP16 lo part turns subnormal and the split loses precision gradually.
//
// The structure follows the FP32 kernel (apply_f32.hip): 4 waves x 3 column
// tiles = 192 columns per workgroup, RT <= 13 16-row tiles of the real
// embedding, the window streamed in chunks of 16 complex rows (32 reals = the
// K of one v_mfma_f32_16x16x32_{bf16,f16}).  Lane (i16, kq) of an operand
// holds reals 8kq..8kq+7 of its row / column (one 16-byte LDS read).  The LS
// chunk is split once, when it is written to LDS.  Per chunk the MFMA phase
// is short (3 RT x 3 products per wave), so the copy of the next chunk's
// filter parts (global-to-LDS, into the other of two buffers) is issued as
// soon as the wave has read its LS operands, ahead of all the chunk's MFMAs.
#include "chunk_io.h"
#include "dft.h"
#include "split.h"

namespace lmmse {

struct SplitArgs {
    const float4* whi;     // hi parts of the real embedding (16-byte units of 8 halves)
    const float4* wlo;     // lo parts (FP16: scaled by 2^11)
    const int* starts;
    const int* classes;
    const float2* x;
    const float2* pilots;
    float2* out;
    long long ncols;
    long long n_tiles;
    int N, B, Wn, G16, Rpad, nb, rgroups;
    int vec_store;
    float invK;            // 1/K times the input scale (fused path)
    float in_scale;        // input scale (unfused path)
    float out_scale;       // 1 / input scale (FP16: times 2^-11)
    int* status;           // plan status word (FP16 range reports)
};

// LS chunk parts in LDS, slot-major: 16-byte slot kq (complex rows
// 4kq..4kq+3) of column c at kq * kXP + c; complex row r of column c is the
// 32-bit word 4 (kq kXP + c) + (r & 3).
__device__ __forceinline__ int xw_at(int c, int r) { return 4 * ((r >> 2) * kXP + c) + (r & 3); }

// LS values of chunk cc, split into hi / lo parts, into LDS.
template <int KF, bool FP16>
__device__ __forceinline__ void split_store_ls(const SplitArgs& a, int tid, int cc,
                                               const RawRegs<KF>& R, uint32_t* xh, uint32_t* xl,
                                               const float2* pl, bool& bad) {
    using CR = RawRegs<KF>;
#pragma unroll
    for (int u = 0; u < CR::TX; ++u) {
        const int i = tid + u * kThreads;
        if (i >= CR::NPAIR) continue;
        const int cq = i >> 4, r = i & 15;
        if constexpr (KF == 0) {
            uint32_t h, l;
            const float2 v = make_float2(R.v[u][0].x * a.in_scale, R.v[u][0].y * a.in_scale);
            if constexpr (FP16) bad |= !f16_in_range(v);
            split_c<FP16>(v, h, l);
            xh[xw_at(cq, r)] = h;
            xl[xw_at(cq, r)] = l;
        } else {
            // rows past the window are scaled by 0 rather than branched
            // around: a branch per user would wait for each pilot read in turn
            const float s = cc * 16 + r < a.Wn ? a.invK : 0.f;
            float2 p[KF];
#pragma unroll
            for (int k = 0; k < KF; ++k) p[k] = pl[k * 16 + r];
            float2 z[KF];
            Dft<KF>::run(R.v[u], z, nullptr);
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                float2 h = cmulc(z[k], p[k]);
                h = make_float2(h.x * s, h.y * s);
                if constexpr (FP16) bad |= !f16_in_range(h);
                uint32_t hh, ll;
                split_c<FP16>(h, hh, ll);
                xh[xw_at(cq * KF + k, r)] = hh;
                xl[xw_at(cq * KF + k, r)] = ll;
            }
        }
    }
}

// Odd blocks stream their window backwards (rev), so that neighbouring
// blocks read the halo they share at about the same time, while it is in L2.
struct SplitCtx {
    const SplitArgs& a;
    size_t wofs0;      // bank offset (16-byte units) of chunk 0 of this row group
    size_t cstride;    // bank offset between consecutive chunks
    long long c0;
    int s0, nchunks, rev, tid, wave, lane, l16, kq;
    __device__ int ch(int step) const { return rev ? nchunks - 1 - step : step; }
};

// One chunk: chunk cc+1's pilots (registers) and chunk cc's split LS values
// into LDS, chunk cc+1's raw inputs into registers, barrier, this wave's LS
// operands from LDS, then the copy of chunk cc+1's filter parts into wnext
// and chunk cc+2's pilots into registers, the chunk's MFMAs (reading only
// wcur, which the compiler can tell from wnext), wait for this wave's loads,
// barrier.
template <int RT, int KF, bool FP16>
__device__ __forceinline__ void split_step(const SplitCtx& x, int cc, float4* xh4, float4* xl4,
                                           float2* pl, float4* wcur, float4* wnext,
                                           floatx4 (&acc)[RT][kCT], RawRegs<KF>& raw,
                                           PilotRegs<KF>& pr, bool& bad) {
    constexpr int NS = PilotRegs<KF>::NS;
    if constexpr (KF > 0)
        if (cc + 1 < x.nchunks) store_pil<KF>(pr, pl + ((cc + 1) & 1) * NS, x.tid);
    split_store_ls<KF, FP16>(x.a, x.tid, x.ch(cc), raw, reinterpret_cast<uint32_t*>(xh4),
                             reinterpret_cast<uint32_t*>(xl4), pl + (cc & 1) * NS, bad);
    if (cc + 1 < x.nchunks) load_raw<KF>(x.a, x.tid, x.ch(cc + 1), x.s0, x.c0, raw);
    __syncthreads();
    float4 bh[kCT], bl[kCT];
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) {
        const int c = (x.wave * kCT + ct) * 16 + x.l16;
        bh[ct] = xh4[x.kq * kXP + c];
        bl[ct] = xl4[x.kq * kXP + c];
    }
    if (cc + 1 < x.nchunks) {
        const size_t o = x.wofs0 + (size_t)x.ch(cc + 1) * x.cstride;
        dma_copy<RT * 64>(x.a.whi + o, wnext, x.wave, x.lane);
        dma_copy<RT * 64>(x.a.wlo + o, wnext + RT * 64, x.wave, x.lane);
        if constexpr (KF > 0)
            if (cc + 2 < x.nchunks) load_pil<KF>(x.a, x.s0, x.ch(cc + 2), x.tid, pr);
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int wi = x.kq * RT * 16 + rt * 16 + x.l16;
        const float4 ahi = wcur[wi], alo = wcur[RT * 64 + wi];
        const float4 a0 = FP16 ? scale2048_f16(ahi) : ahi;
        // three independent column tiles between dependent products
#pragma unroll
        for (int ct = 0; ct < kCT; ++ct) acc[rt][ct] = mma<FP16>(a0, bh[ct], acc[rt][ct]);
#pragma unroll
        for (int ct = 0; ct < kCT; ++ct) acc[rt][ct] = mma<FP16>(alo, bh[ct], acc[rt][ct]);
#pragma unroll
        for (int ct = 0; ct < kCT; ++ct) acc[rt][ct] = mma<FP16>(ahi, bl[ct], acc[rt][ct]);
    }
    wait_vm();
    __syncthreads();
}

template <int RT, int KF>
constexpr int split_min_blocks() { return (KF == 24 || (RT >= 13 && KF <= 2)) ? 1 : 2; }

// 4 waves x 3 column tiles, RT <= 13 row tiles.  Two workgroups per CU where
// the registers allow it (K = 24 and the tallest unfused / K <= 2 variants
// run one per CU rather than spill).
template <int RT, int KF, bool FP16>
__global__ __launch_bounds__(kThreads, (split_min_blocks<RT, KF>())) void apply_split_kernel(
    SplitArgs a) {
    constexpr int NS = PilotRegs<KF>::NS;
    __shared__ float4 xh4[4 * kXP];        // LS chunk, hi parts: [kq][col]
    __shared__ float4 xl4[4 * kXP];        // lo parts
    __shared__ float4 wA[2 * RT * 64];     // filter chunks, even / odd: [hi, lo][kq][row]
    __shared__ float4 wB[2 * RT * 64];
    __shared__ float2 pl[2 * NS];          // pilot slices of two chunks

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave
    long long t = xcd_remap(blockIdx.x, a.n_tiles);
    const int rg = (int)(t % a.rgroups);
    t /= a.rgroups;
    const int b = (int)(t % a.nb);
    const int cls = a.classes[b];
    const SplitCtx x{a,
                     ((size_t)cls * a.G16 * a.rgroups + rg) * (RT * 64),
                     (size_t)a.rgroups * (RT * 64),
                     (t / a.nb) * kCols,
                     a.starts[b],
                     a.G16,
                     b & 1,
                     tid,
                     wave,
                     lane,
                     lane & 15,
                     lane >> 4};

    floatx4 acc[RT][kCT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < kCT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};

    PilotRegs<KF> pr;
    RawRegs<KF> raw;
    const size_t o0 = x.wofs0 + (size_t)x.ch(0) * x.cstride;
    dma_copy<RT * 64>(a.whi + o0, wA, wave, lane);
    dma_copy<RT * 64>(a.wlo + o0, wA + RT * 64, wave, lane);
    if constexpr (KF > 0) {
        load_pil<KF>(a, x.s0, x.ch(0), tid, pr);
        store_pil<KF>(pr, pl, tid);
        if (x.nchunks > 1) load_pil<KF>(a, x.s0, x.ch(1), tid, pr);
    }
    load_raw<KF>(a, tid, x.ch(0), x.s0, x.c0, raw);
    wait_vm();
    __syncthreads();
    bool bad = false;
    for (int cc = 0; cc < x.nchunks; cc += 2) {
        split_step<RT, KF, FP16>(x, cc, xh4, xl4, pl, wA, wB, acc, raw, pr, bad);
        if (cc + 1 < x.nchunks)
            split_step<RT, KF, FP16>(x, cc + 1, xh4, xl4, pl, wB, wA, acc, raw, pr, bad);
    }
    if constexpr (FP16) report_range(bad, a.status);

    const int l16 = x.l16, kq = x.kq;
    const bool vec = a.vec_store != 0;
    const float sc = a.out_scale;
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) {
        const long long col = x.c0 + (wave * kCT + ct) * 16 + l16;
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
    const dim3 grid((unsigned)a.n_tiles), block(kThreads);
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
    a.whi = reinterpret_cast<const float4*>(p.whi);
    a.wlo = reinterpret_cast<const float4*>(p.wlo);
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
    a.invK = p.in_scale / (float)p.d.K;
    a.in_scale = p.in_scale;
    a.out_scale = (fp16 ? 1.0f / 2048.0f : 1.0f) / p.in_scale;
    a.status = p.status;
    a.vec_store = (((a.N | a.B) & 1) == 0 && ((uintptr_t)out & 15) == 0) ? 1 : 0;
    const long long ctiles = (a.ncols + kCols - 1) / kCols;
    a.n_tiles = ctiles * p.nb * p.rgroups;
    if (a.n_tiles == 0) return hipSuccess;
    const int kf = fused ? p.d.K : 0;
    return fp16 ? launch_split_t<true>(a, p.RT, kf, st) : launch_split_t<false>(a, p.RT, kf, st);
}

}  // namespace lmmse
