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
// window is streamed in chunks of 16 complex rows (two groups of 8).  Per
// chunk the workgroup puts the LS values into LDS (from H_LS, or made on the
// fly from the pilot symbols: one thread per (antenna, subcarrier) undoes the
// cover code of y[s,m,0..K-1,n] with a K-point DFT and multiplies by
// conj(x_k[n]) / K), then every wave runs RT x 3 x 8 MFMAs against the
// chunk's filter rows.  Memory latency is kept off the matrix cores: the raw
// inputs of chunk c+1 are loaded into registers before the MFMAs of chunk c;
// the filter rows of chunk c+1 are copied global-to-LDS into the other of two
// buffers, and the pilot slice of chunk c+2 loaded, halfway through them;
// two workgroups share a CU.  The block index runs fastest over consecutive
// tiles and tiles are remapped so that each XCD takes a contiguous range: the
// overlapping windows of neighbouring blocks of a column group are read
// through the same L2.
#include "chunk_io.h"
#include "dft.h"

namespace lmmse {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Block b of the launch reads x[col][starts[b] + j], j < Wn (the
// contraction), and writes out[col][ostarts[b] + o], o < B; the forward pass
// has starts = window starts, ostarts = b*B, and the backward dX pass the
// transposed roles with the W^H bank.  The launch covers blocks pass,
// pass + P, ... (nbp of them).
struct ApplyArgs {
    const float4* wbank;
    const int* starts;
    const int* ostarts;
    const int* classes;
    const float2* x;       // H_LS [cols][N] (unfused) or y [S*M][K][N] (fused)
    const float2* pilots;  // [K][N] (fused only)
    float2* out;           // [cols][N]
    long long ncols;       // S*M*K
    long long n_tiles;
    int N, B, Wn, G16, Rpad, nbp, pass, P, rgroups;
    int vec_store;         // out offsets even and out 16-byte aligned: float4 stores
    int accumulate;        // out += (read-add-write) instead of out =
    float invK;
};

__device__ __forceinline__ float f4c(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// LS chunk in LDS: slot f (complex rows 2f, 2f+1, one float4) of column c.
__device__ __forceinline__ int xs4_at(int c, int f) { return f * kXP + c; }
__device__ __forceinline__ int xs2_at(int c, int r) { return 2 * xs4_at(c, r >> 1) + (r & 1); }

// LS values of chunk cc into LDS: straight (unfused) or despread (fused).
template <int KF>
__device__ __forceinline__ void store_ls(const ApplyArgs& a, int tid, int cc, const RawRegs<KF>& R,
                                         float2* xs2, const float2* pl) {
    using CR = RawRegs<KF>;
#pragma unroll
    for (int u = 0; u < CR::TX; ++u) {
        const int i = tid + u * kThreads;
        if (i >= CR::NPAIR) continue;
        const int cq = i >> 4, r = i & 15;
        if constexpr (KF == 0) {
            xs2[xs2_at(cq, r)] = R.v[u][0];
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
                const float2 h = cmulc(z[k], p[k]);
                xs2[xs2_at(cq * KF + k, r)] = make_float2(h.x * s, h.y * s);
            }
        }
    }
}

// LS operands of one group of 8 complex window rows for this wave's 3
// column tiles.
__device__ __forceinline__ void load_xv(float4 (&xv)[kCT], const float4* xs4, int gg, int wave,
                                        int l16, int q) {
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) xv[ct] = xs4[xs4_at((wave * kCT + ct) * 16 + l16, 4 * gg + q)];
}

// One group of 8 complex window rows: 4 k-steps x RT x 3 MFMAs per wave.
// ws4 holds the chunk's filter rows as [gg][q][row].
template <int RT>
__device__ __forceinline__ void mfma_group(floatx4 (&acc)[RT][kCT], const float4 (&xv)[kCT],
                                           const float4* ws4, int gg, int l16, int q) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const float4 av = ws4[gg * RT * 64 + q * RT * 16 + rt * 16 + l16];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int ct = 0; ct < kCT; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(f4c(av, i), f4c(xv[ct], i),
                                                                   acc[rt][ct], 0, 0, 0);
    }
}

// Filter rows of chunk cc of this workgroup's row group into LDS: two runs
// of RT*64 float4 (one per group of 8 window rows), contiguous in the bank.
template <int RT>
__device__ __forceinline__ void copy_w(const float4* wsrc, size_t gstride, int cc, int wave,
                                       int lane, float4* wdst) {
    dma_copy<RT * 64>(wsrc + (size_t)(2 * cc) * gstride, wdst, wave, lane);
    dma_copy<RT * 64>(wsrc + (size_t)(2 * cc + 1) * gstride, wdst + RT * 64, wave, lane);
}

// Per-workgroup constants of the filtering loop.
// Odd blocks stream their window backwards (rev): the halo a block shares
// with each neighbour is then read by both at about the same time, while it
// is still in L2.
struct ChunkCtx {
    const ApplyArgs& a;
    const float4* wsrc;
    size_t gstride;
    long long c0;
    int s0, nchunks, rev, tid, wave, lane, l16, q;
    __device__ int ch(int step) const { return rev ? nchunks - 1 - step : step; }
};

// One chunk: chunk cc+1's pilots (held in registers) and chunk cc's LS values
// into LDS, chunk cc+1's raw inputs into registers, barrier, the MFMAs of
// the first group, the copy of chunk cc+1's filter rows into wnext and chunk
// cc+2's pilots into registers, the MFMAs of the second group, wait for this
// wave's loads, barrier.  wcur / wnext name the two LDS filter buffers
// directly, so the compiler sees that the copy into one does not touch the
// other and adds no wait before the reads of wcur; the LS operands of the
// second group are read before the copy is issued (the compiler cannot tell
// xs4 from wnext and would wait for the copy before reading them).
template <int RT, int KF>
__device__ __forceinline__ void chunk_step(const ChunkCtx& x, int cc, float4* xs4, float2* pl,
                                           float4* wcur, float4* wnext, floatx4 (&acc)[RT][kCT],
                                           RawRegs<KF>& raw, PilotRegs<KF>& pr) {
    constexpr int NS = PilotRegs<KF>::NS;
    if constexpr (KF > 0)
        if (cc + 1 < x.nchunks) store_pil<KF>(pr, pl + ((cc + 1) & 1) * NS, x.tid);
    store_ls<KF>(x.a, x.tid, x.ch(cc), raw, reinterpret_cast<float2*>(xs4), pl + (cc & 1) * NS);
    if (cc + 1 < x.nchunks) load_raw<KF>(x.a, x.tid, x.ch(cc + 1), x.s0, x.c0, raw);
    __syncthreads();
    float4 xv[kCT];
    load_xv(xv, xs4, 0, x.wave, x.l16, x.q);
    mfma_group<RT>(acc, xv, wcur, 0, x.l16, x.q);
    load_xv(xv, xs4, 1, x.wave, x.l16, x.q);
    if (cc + 1 < x.nchunks) {
        copy_w<RT>(x.wsrc, x.gstride, x.ch(cc + 1), x.wave, x.lane, wnext);
        if constexpr (KF > 0)
            if (cc + 2 < x.nchunks) load_pil<KF>(x.a, x.s0, x.ch(cc + 2), x.tid, pr);
    }
    // the second group of the last chunk may lie wholly past the window
    if (16 * x.ch(cc) + 8 < x.a.Wn) mfma_group<RT>(acc, xv, wcur, 1, x.l16, x.q);
    wait_vm();
    __syncthreads();
}

// RT row tiles x 3 column tiles per wave, 4 waves.  Two workgroups per CU
// where registers and LDS allow it (tall row groups and K = 24 run one per
// CU rather than spill).
template <int RT, int KF>
constexpr int min_blocks() { return (RT <= 13 && KF != 24) ? 2 : 1; }

template <int RT, int KF>
__global__ __launch_bounds__(kThreads, (min_blocks<RT, KF>())) void apply_f32_kernel(ApplyArgs a) {
    constexpr int NS = PilotRegs<KF>::NS;
    __shared__ float4 xs4[8 * kXP];           // LS chunk: [slot][col]
    __shared__ float4 wA[2 * RT * 64];        // filter chunks, even / odd: [gg][q][row]
    __shared__ float4 wB[2 * RT * 64];
    __shared__ float2 pl[2 * NS];             // pilot slices of two chunks

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave
    long long t = xcd_remap(blockIdx.x, a.n_tiles);
    const int rg = (int)(t % a.rgroups);
    t /= a.rgroups;
    const int b = a.pass + a.P * (int)(t % a.nbp);
    const int cls = a.classes[b];
    const ChunkCtx x{a,
                     a.wbank + ((size_t)cls * 2 * a.G16 * a.rgroups + rg) * (RT * 64),
                     (size_t)a.rgroups * (RT * 64),
                     (t / a.nbp) * kCols,
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
    copy_w<RT>(x.wsrc, x.gstride, x.ch(0), wave, lane, wA);
    if constexpr (KF > 0) {
        load_pil<KF>(a, x.s0, x.ch(0), tid, pr);
        store_pil<KF>(pr, pl, tid);
        if (x.nchunks > 1) load_pil<KF>(a, x.s0, x.ch(1), tid, pr);
    }
    load_raw<KF>(a, tid, x.ch(0), x.s0, x.c0, raw);
    wait_vm();
    __syncthreads();
    for (int cc = 0; cc < x.nchunks; cc += 2) {
        chunk_step<RT, KF>(x, cc, xs4, pl, wA, wB, acc, raw, pr);
        if (cc + 1 < x.nchunks) chunk_step<RT, KF>(x, cc + 1, xs4, pl, wB, wA, acc, raw, pr);
    }

    // lane (l16, q) of tile (rt, ct) holds real rows 16rt + 4q .. +3 of its
    // column: complex outputs o, o+1 of the block
    const int l16 = x.l16, q = x.q;
    const bool vec = a.vec_store != 0;
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) {
        const long long col = x.c0 + (wave * kCT + ct) * 16 + l16;
        if (col >= a.ncols) continue;
        float2* op = a.out + col * a.N + a.ostarts[b];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int o = (((rg * RT + rt) * 16) + 4 * q) >> 1;
            const floatx4 v = acc[rt][ct];
            if (a.accumulate) {
                if (o < a.B) {
                    const float2 c0v = op[o];
                    op[o] = make_float2(c0v.x + v[0], c0v.y + v[1]);
                }
                if (o + 1 < a.B) {
                    const float2 c1v = op[o + 1];
                    op[o + 1] = make_float2(c1v.x + v[2], c1v.y + v[3]);
                }
            } else if (o + 1 < a.B) {
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

static hipError_t launch_args(const ApplyArgs& a, int RT, int kf, hipStream_t st) {
    const dim3 grid((unsigned)a.n_tiles);
#define LMMSE_AF(R, KK)                                                                  \
    case R:                                                                              \
        hipLaunchKernelGGL((apply_f32_kernel<R, KK>), grid, dim3(kThreads), 0, st, a);   \
        break;
#define LMMSE_AFK(KK)                                                                    \
    case KK:                                                                             \
        switch (RT) {                                                                    \
            LMMSE_AF(1, KK) LMMSE_AF(2, KK) LMMSE_AF(4, KK) LMMSE_AF(8, KK)              \
            LMMSE_AF(9, KK) LMMSE_AF(13, KK) LMMSE_AF(15, KK) LMMSE_AF(17, KK)           \
            default: return hipErrorInvalidValue;                                        \
        }                                                                                \
        break;
    switch (kf) {
        case 0:
            switch (RT) {
                LMMSE_AF(1, 0) LMMSE_AF(2, 0) LMMSE_AF(4, 0) LMMSE_AF(8, 0) LMMSE_AF(9, 0)
                LMMSE_AF(10, 0) LMMSE_AF(13, 0) LMMSE_AF(15, 0) LMMSE_AF(17, 0)
                default: return hipErrorInvalidValue;
            }
            break;
        LMMSE_AFK(1) LMMSE_AFK(2) LMMSE_AFK(4) LMMSE_AFK(12) LMMSE_AFK(24)
        default:
            return hipErrorInvalidValue;
    }
#undef LMMSE_AFK
#undef LMMSE_AF
    return hipGetLastError();
}

hipError_t launch_apply_f32(const Plan& p, int slots, const float2* x, const float2* pilots,
                            bool fused, float2* out, hipStream_t st) {
    ApplyArgs a;
    a.wbank = p.wf32;
    a.starts = p.d_starts;
    a.ostarts = p.d_bstarts;
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
    a.nbp = p.nb;
    a.pass = 0;
    a.P = 1;
    a.rgroups = p.rgroups;
    a.accumulate = 0;
    a.invK = 1.0f / (float)p.d.K;
    a.vec_store = (((a.N | a.B) & 1) == 0 && ((uintptr_t)out & 15) == 0) ? 1 : 0;
    const long long ctiles = (a.ncols + kCols - 1) / kCols;
    a.n_tiles = ctiles * p.nb * p.rgroups;
    if (a.n_tiles == 0) return hipSuccess;
    return launch_args(a, p.RT, fused ? p.d.K : 0, st);
}

// Row tiles of the transposed product: padded tiles, charged 5% per row group
// (each group re-reads its input window and redoes the staging).
void transposed_row_tiles(int out_len, int& RT, int& rgroups) {
    static const int cand[] = {1, 2, 4, 8, 9, 10, 13, 15, 17};
    const int T = (2 * out_len + 15) / 16;
    double best = -1.0;
    for (int rt : cand) {
        const int g = (T + rt - 1) / rt;
        const double cost = (double)g * rt * (1.0 + 0.05 * g);
        if (best < 0.0 || cost < best) {
            best = cost;
            RT = rt;
            rgroups = g;
        }
    }
}

hipError_t launch_apply_f32_transposed(const Plan& p, int slots, const float4* bank, int RT,
                                       int rgroups, int pass, int P, const float2* g, float2* dx,
                                       int accumulate, hipStream_t st) {
    ApplyArgs a;
    a.wbank = bank;
    a.starts = p.d_bstarts;
    a.ostarts = p.d_starts;
    a.classes = p.d_classes;
    a.x = g;
    a.pilots = nullptr;
    a.out = dx;
    a.ncols = (long long)slots * p.d.M * p.d.K;
    a.N = p.d.N;
    a.B = p.d.Wn;
    a.Wn = p.d.B;
    a.G16 = (p.d.B + 15) / 16;
    a.Rpad = RT * 16 * rgroups;
    a.nbp = (p.nb - pass + P - 1) / P;
    a.pass = pass;
    a.P = P;
    a.rgroups = rgroups;
    a.accumulate = accumulate;
    a.invK = 1.0f;
    a.vec_store = 0;
    const long long ctiles = (a.ncols + kCols - 1) / kCols;
    a.n_tiles = ctiles * a.nbp * rgroups;
    if (a.n_tiles <= 0 || a.nbp <= 0) return hipSuccess;
    return launch_args(a, RT, 0, st);
}

}  // namespace lmmse
