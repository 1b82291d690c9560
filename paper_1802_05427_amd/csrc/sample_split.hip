// Split-precision filtering of the sample-covariance path (eq. 12 per
// (slot, user, block)): Hhat[s, m, k, O_b] = W_(s,k,b) h_ls[s, m, k, I_b] for
// the M antennas, with the products hi_W hi_X + lo_W hi_X + hi_W lo_X on
// v_mfma_f32_16x16x32_{f16,bf16} and FP32 accumulation (split rules as in
// apply_split.hip: FP16 lo parts and the hi_W hi_X product carry 2^11, undone
// at the store).
//
// Workgroup: 4 waves x 2 column tiles = 128 antennas of one window, RT
// 16-row tiles of the real embedding of one row group, the window streamed in
// chunks of 16 complex rows (the 32 reals of one MFMA's K).
//  * filter parts: the design writes them compact and chunk-major, packed
//    (re, im) 16-bit pairs, the 16 columns of one chunk of all B rows of a
//    window in one contiguous block (split_w_index).  A chunk's rows are
//    copied global-to-LDS (four 16-byte slots of 4 complex entries per row and
//    part, whole 128-byte lines) into one of two buffers; lane (i16, kq) of a tile reads slot kq of its output row and
//    forms its embedded operand in registers: (re, -im) pairs for the real
//    output row, (im, re) for the imaginary one;
//  * LS values: one chunk ahead in registers, split into hi / lo when written
//    to LDS, slot-major like the FP32 kernel's.
#include "internal.h"
#include "split.h"

namespace lmmse {

struct SampleSplitArgs {
    const float2* hls;
    const uint32_t* whi;   // per window B x Wq, chunk-major (Wq = Wn rounded up to 16)
    const uint32_t* wlo;
    const int* starts;
    float2* out;
    long long n_tiles;
    int M, K, N, B, Wn, Wq, nb, rgroups, G16, cgroups;
    float in_scale;    // power-of-two input scale applied before the split
    float out_scale;   // its inverse (FP16: times 2^-11)
    int* status;       // plan status word (FP16 range reports)
};

constexpr int sCT = 2;                  // column tiles per wave
constexpr int sThreads = 256;           // 4 waves
constexpr int sCols = 16 * sCT * 4;     // 128 antennas per workgroup
constexpr int sXP = sCols + 1;          // LS chunk stride in 16-byte slots (slot-major)

// LS part word of complex row r (0..15) of column c: slot r / 4, word r % 4.
__device__ __forceinline__ int sx_at(int c, int r) { return 4 * ((r >> 2) * sXP + c) + (r & 3); }

// Slots per part buffer: 8 RT rows x 4 slots, rounded up to whole 64-slot
// runs of the direct copies (the extra slots hold clamped rows, never read).
template <int RT>
constexpr int ss_slots() { return (RT * 32 + 63) / 64 * 64; }

// Filter parts of chunk cc for output rows o0 .. o0 + 8 RT - 1 into LDS: slot
// 4 ol + (kq ^ (ol & 3)) of each part buffer holds entries 16 cc + 4 kq ..
// +3 of row o0 + ol, read from the chunk's contiguous block.  Rows past B
// repeat row B - 1 (discarded outputs); the columns past Wn are zero.
template <int RT>
__device__ __forceinline__ void split_copy_w(const uint32_t* whi, const uint32_t* wlo, int B,
                                             int o0, int cc, int wave, int lane, float4* dhi,
                                             float4* dlo) {
    constexpr int NV = ss_slots<RT>();
#pragma unroll
    for (int part = 0; part < 2; ++part)
#pragma unroll
        for (int u = 0; u < (NV + sThreads - 1) / sThreads; ++u) {
            const int base = u * sThreads + wave * 64;
            if (base < NV) {
                const int sl = base + lane, ol = sl >> 2, kq = (sl & 3) ^ (ol & 3);
                const int o = min(o0 + ol, B - 1);
                const uint32_t* src = (part ? wlo : whi) + (unsigned)((cc * B + o) * 16 + 4 * kq);
                float4* dst = (part ? dlo : dhi) + base;
                __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst,
                                                 16, 0, 0);
            }
        }
}

// Embedded operand of an output row from its 4 packed complex entries:
// real row (im = 0): (re, -im) per entry; imaginary row: (im, re).
__device__ __forceinline__ float4 embed_row(const float4& w, int im) {
    const uint32_t* u = reinterpret_cast<const uint32_t*>(&w);
    uint32_t r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        r[i] = im ? __builtin_amdgcn_alignbit(u[i], u[i], 16) : (u[i] ^ 0x80000000u);
    return make_float4(__builtin_bit_cast(float, r[0]), __builtin_bit_cast(float, r[1]),
                       __builtin_bit_cast(float, r[2]), __builtin_bit_cast(float, r[3]));
}

struct SampleSplitRaw {
    float2 v[8];
};

__device__ __forceinline__ void ss_load_x(const SampleSplitArgs& a, const float2* xbase,
                                          long long xstride, int m0, int cc, int tid,
                                          SampleSplitRaw& R) {
    const int r = tid & 15, c0 = tid >> 4, j = 16 * cc + r;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int m = m0 + c0 + 16 * u;
        R.v[u] = (j < a.Wn && m < a.M) ? xbase[m * xstride + j] : make_float2(0.f, 0.f);
    }
}

template <bool FP16>
__device__ __forceinline__ void ss_store_x(const SampleSplitRaw& R, int tid, uint32_t* xh,
                                           uint32_t* xl, float in_scale, bool& bad) {
    const int r = tid & 15, c0 = tid >> 4;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        uint32_t h, l;
        const float2 v = make_float2(R.v[u].x * in_scale, R.v[u].y * in_scale);
        if constexpr (FP16) bad |= !f16_in_range(v);
        split_c<FP16>(v, h, l);
        xh[sx_at(c0 + 16 * u, r)] = h;
        xl[sx_at(c0 + 16 * u, r)] = l;
    }
}

struct SampleSplitCtx {
    const SampleSplitArgs& a;
    const float2* xbase;
    const uint32_t* whi;
    const uint32_t* wlo;
    long long xstride;
    int m0, o0, nchunks, tid, wave, lane, l16, kq;
};

// One chunk: LS parts into LDS, next chunk's LS values into registers,
// barrier, this wave's LS operands, the copy of the next chunk's filter parts
// into the other buffers, the MFMAs (RT x 2 x 3 per wave), wait, barrier.
template <int RT, bool FP16>
__device__ __forceinline__ void ss_step(const SampleSplitCtx& x, int cc, uint32_t* xh, uint32_t* xl,
                                        const float4* hcur, const float4* lcur, float4* hnext,
                                        float4* lnext, floatx4 (&acc)[RT][sCT], SampleSplitRaw& raw,
                                        bool& bad) {
    ss_store_x<FP16>(raw, x.tid, xh, xl, x.a.in_scale, bad);
    if (cc + 1 < x.nchunks) ss_load_x(x.a, x.xbase, x.xstride, x.m0, cc + 1, x.tid, raw);
    __syncthreads();
    float4 bh[sCT], bl[sCT];
    const float4* xh4 = reinterpret_cast<const float4*>(xh);
    const float4* xl4 = reinterpret_cast<const float4*>(xl);
#pragma unroll
    for (int ct = 0; ct < sCT; ++ct) {
        const int c = (x.wave * sCT + ct) * 16 + x.l16;
        bh[ct] = xh4[x.kq * sXP + c];
        bl[ct] = xl4[x.kq * sXP + c];
    }
    if (cc + 1 < x.nchunks)
        split_copy_w<RT>(x.whi, x.wlo, x.a.B, x.o0, cc + 1, x.wave, x.lane, hnext, lnext);
    const int im = x.l16 & 1;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int ol = 8 * rt + (x.l16 >> 1), sl = 4 * ol + (x.kq ^ (ol & 3));
        const float4 ah = embed_row(hcur[sl], im);
        const float4 al = embed_row(lcur[sl], im);
        const float4 a0 = FP16 ? scale2048_f16(ah) : ah;
#pragma unroll
        for (int ct = 0; ct < sCT; ++ct) {
            acc[rt][ct] = mma<FP16>(a0, bh[ct], acc[rt][ct]);
            acc[rt][ct] = mma<FP16>(al, bh[ct], acc[rt][ct]);
            acc[rt][ct] = mma<FP16>(ah, bl[ct], acc[rt][ct]);
        }
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies have landed
    __syncthreads();
}

template <int RT, bool FP16>
__global__ __launch_bounds__(sThreads, 2) void apply_sample_split_kernel(SampleSplitArgs a) {
    __shared__ uint32_t xh[4 * 4 * sXP];   // 4 slots x sXP columns x 4 words
    __shared__ uint32_t xl[4 * 4 * sXP];
    __shared__ float4 hA[ss_slots<RT>()];
    __shared__ float4 lA[ss_slots<RT>()];
    __shared__ float4 hB[ss_slots<RT>()];
    __shared__ float4 lB[ss_slots<RT>()];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    long long t = blockIdx.x;
    const int rg = (int)(t % a.rgroups);
    t /= a.rgroups;
    const int cg = (int)(t % a.cgroups);
    t /= a.cgroups;
    const int b = (int)(t % a.nb);
    const long long sk = t / a.nb;
    const int k = (int)(sk % a.K);
    const long long s = sk / a.K;
    const long long wofs = ((sk * a.nb + b) * a.B) * (long long)a.Wq;
    const SampleSplitCtx x{a,
                           a.hls + ((s * a.M) * a.K + k) * (long long)a.N + a.starts[b],
                           a.whi + wofs,
                           a.wlo + wofs,
                           (long long)a.K * a.N,
                           cg * sCols,
                           rg * RT * 8,
                           a.G16,
                           tid,
                           wave,
                           lane,
                           lane & 15,
                           lane >> 4};
    floatx4 acc[RT][sCT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < sCT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    SampleSplitRaw raw;
    split_copy_w<RT>(x.whi, x.wlo, a.B, x.o0, 0, wave, lane, hA, lA);
    ss_load_x(a, x.xbase, x.xstride, x.m0, 0, tid, raw);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    bool bad = false;
    for (int cc = 0; cc < x.nchunks; cc += 2) {
        ss_step<RT, FP16>(x, cc, xh, xl, hA, lA, hB, lB, acc, raw, bad);
        if (cc + 1 < x.nchunks) ss_step<RT, FP16>(x, cc + 1, xh, xl, hB, lB, hA, lA, acc, raw, bad);
    }
    if constexpr (FP16) report_range(bad, a.status);
    // lane (l16, kq) of tile (rt, ct) holds real rows 16 rt + 4 kq .. +3 of its
    // column: complex outputs o, o + 1 of the block
    const int l16 = x.l16, q = x.kq;
    const float sc = a.out_scale;
#pragma unroll
    for (int ct = 0; ct < sCT; ++ct) {
        const int m = x.m0 + (wave * sCT + ct) * 16 + l16;
        if (m >= a.M) continue;
        float2* op = a.out + ((s * a.M + m) * a.K + k) * (long long)a.N + (long long)b * a.B;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int o = (((rg * RT + rt) * 16) + 4 * q) >> 1;
            const floatx4 v = acc[rt][ct];
            if (o < a.B) op[o] = make_float2(v[0] * sc, v[1] * sc);
            if (o + 1 < a.B) op[o + 1] = make_float2(v[2] * sc, v[3] * sc);
        }
    }
}

hipError_t launch_apply_sample_split(const Plan& p, long long nmat, const float2* hls,
                                     const uint32_t* whi, const uint32_t* wlo, float2* out,
                                     hipStream_t st) {
    if (nmat == 0) return hipSuccess;
    SampleSplitArgs a{};
    a.hls = hls;
    a.whi = whi;
    a.wlo = wlo;
    a.starts = p.d_starts;
    a.out = out;
    a.M = p.d.M;
    a.K = p.d.K;
    a.N = p.d.N;
    a.B = p.d.B;
    a.Wn = p.d.Wn;
    a.Wq = (p.d.Wn + 15) & ~15;
    a.nb = p.nb;
    a.rgroups = p.srgroups;
    a.G16 = p.G16;
    a.cgroups = (p.d.M + sCols - 1) / sCols;
    a.n_tiles = nmat * a.cgroups * p.srgroups;
    const bool fp16 = p.d.precision == LMMSE_FP16X3;
    a.in_scale = p.in_scale;
    a.out_scale = (fp16 ? 1.0f / 2048.0f : 1.0f) / p.in_scale;
    a.status = p.status;
    const dim3 grid((unsigned)a.n_tiles), block(sThreads);
#define LMMSE_SS(R)                                                                        \
    case R:                                                                                \
        if (fp16)                                                                          \
            hipLaunchKernelGGL((apply_sample_split_kernel<R, true>), grid, block, 0, st, a);  \
        else                                                                               \
            hipLaunchKernelGGL((apply_sample_split_kernel<R, false>), grid, block, 0, st, a); \
        break;
    switch (p.sRT) {
        LMMSE_SS(1) LMMSE_SS(2) LMMSE_SS(4) LMMSE_SS(8) LMMSE_SS(9) LMMSE_SS(13) LMMSE_SS(15)
        LMMSE_SS(17)
        default:
            return hipErrorInvalidValue;
    }
#undef LMMSE_SS
    return hipGetLastError();
}

}  // namespace lmmse
