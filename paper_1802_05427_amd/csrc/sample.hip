// Sample-covariance path: per (slot s, user k, block b) the window correlation
// is the raw sample covariance over the M antennas,
//     R = (1/M) sum_m x_m x_m^H,   x_m = h_ls[s, m, k, I_b]  (Wn values),
// and the block filter is W = R_OI (R + lam I)^-1 = (I - lam A^-1)[off_b rows]
// with A = R + lam I (eq. 13 on the block, Sec. IV-B).
//
// sample_design_kernel: one workgroup of 1024 threads per (s, k, b).  The
// matrix is cut into 32 x 32 blocks; only blocks (P, Q) with P >= Q are kept,
// the diagonal ones in full, and thread (tr, tc) = (t % 32, t / 32) holds
// entry (32P + tr, 32Q + tc) of every kept block in registers (n <= 32 NBK).
// R is accumulated in FP64 from the FP32 LS values (the products are exact),
// staged through LDS 16 antennas at a time.  A = R + lam I is then inverted
// in place by the Hermitian sweep, written as one rank-1 update per pivot k:
// with d = A[k][k], c = A[:, k] and w = c - e_k,
//     A <- A - w w^H / d,   then A[k][k] -= 2,
// which gives A[i][j] - c_i conj(c_j)/d off the pivot row and column,
// c_i / d and conj(c_j) / d on them and -1/d at (k, k); after all n pivots
// A holds -A^-1 (Gauss-Jordan elimination without pivoting, safe for a
// positive definite A).  The pivot loop is unrolled over the column blocks,
// so the owners of the next pivot column know at compile time which of their
// registers hold it; they publish it through a double-buffered LDS vector,
// one barrier per pivot.
//
// apply_sample_kernel: Hhat[s, m, k, O_b] = W_(s,k,b) h_ls[s, m, k, I_b] for the
// M antennas (128 per workgroup), on v_mfma_f32_16x16x4f32 with the operand
// order of the fixed path (apply_f32.hip).  The compact complex FP32 filter is
// streamed in 16-row chunks into two LDS buffers by the direct global-to-LDS
// loads, and each MFMA's real-embedded operand is built in registers from one
// 16-byte complex pair.
#include <algorithm>

#include "internal.h"
#include "split.h"

namespace lmmse {

__device__ __forceinline__ double2 dz_mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 dz_mulc(double2 a, double2 b) {   // a * conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

struct SampleArgs {
    const float2* hls;      // [S][M][K][N]
    const double2* r_in;    // optional [mat][Wn][Wn] (row-major), used instead of hls
    double2* r_out;         // optional: R (before lam) [mat][Wn][Wn]
    double2* w64;           // optional: W [mat][B][Wn]
    float2* w32;            // optional: W, B x W16 per window in the chunk-major order of
                            // split_w_index (W16 = Wn rounded up to 16, pad 0)
    double2* ainv;          // optional: A^-1 [mat][Wn][Wn] (row-major, both triangles)
    uint32_t* whi;          // optional: split W, hi parts packed (re, im) 16-bit, chunk-major
    uint32_t* wlo;          // (split_w_index) and lo parts (FP16: scaled by 2^11)
    int split_fp16;         // split format: FP16 (else BF16)
    const int* starts;
    const int* offsets;
    int* status;
    int M, K, N, B, Wn, nb;
    double lam;
    int want_w;
    long long mat0;         // index of the first matrix (error reports)
};

// Entry index of kept block (P, Q), P >= Q.
__host__ __device__ constexpr int blk(int P, int Q) { return P * (P + 1) / 2 + Q; }

// Publish column kn = 32 QN + tn of the current A into cn: rows i >= 32 QN
// from column block QN (owners tc == tn), rows i < 32 QN from row block QN
// (owners tr == tn, conjugated: A[i][kn] = conj(A[kn][i])).
template <int NBK, int QN>
__device__ __forceinline__ void publish_col(const double2 (&A)[NBK * (NBK + 1) / 2], int tn, int tr,
                                            int tc, int n, double2* cn) {
    if (tc == tn) {
#pragma unroll
        for (int P = QN; P < NBK; ++P) {
            const int i = 32 * P + tr;
            if (i < n) cn[i] = A[blk(P, QN)];
        }
    }
    if (tr == tn) {
#pragma unroll
        for (int Q = 0; Q < QN; ++Q) {
            const double2 v = A[blk(QN, Q)];
            cn[32 * Q + tc] = make_double2(v.x, -v.y);
        }
    }
}

template <int NBK>
__global__ __launch_bounds__(1024) void sample_design_kernel(SampleArgs a) {
    constexpr int AM = 16;                     // antennas per LDS chunk
    constexpr int NMAX = 32 * NBK;
    constexpr int NE = NBK * (NBK + 1) / 2;    // kept blocks = entries per thread
    __shared__ float2 xs[AM][NMAX];
    __shared__ double2 cb[2][NMAX];

    const int tid = threadIdx.x, tr = tid & 31, tc = tid >> 5;
    const int n = a.Wn;
    const long long mat = blockIdx.x;
    const int b = (int)(mat % a.nb);
    const long long sk = mat / a.nb;
    const int k = (int)(sk % a.K);
    const long long s = sk / a.K;
    const int st = a.starts[b];
    double lam_s = a.lam, ainv_s = 1.0;   // lam and 1/alpha of the scaled sweep (below)

    double2 A[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) A[e] = make_double2(0.0, 0.0);

    if (a.r_in) {
        const double2* R = a.r_in + mat * n * n;
#pragma unroll
        for (int P = 0; P < NBK; ++P)
#pragma unroll
            for (int Q = 0; Q <= P; ++Q) {
                const int i = 32 * P + tr, j = 32 * Q + tc;
                if (i < n && j < n) A[blk(P, Q)] = R[(long long)i * n + j];
            }
    } else {
        const double invM = 1.0 / a.M;
        const float2* xrow = a.hls + ((s * a.M) * a.K + k) * (long long)a.N + st;   // antenna 0
        const long long mstride = (long long)a.K * a.N;
        for (int m0 = 0; m0 < a.M; m0 += AM) {
            for (int e = tid; e < AM * NMAX; e += 1024) {
                const int mm = e / NMAX, j = e - mm * NMAX;
                const int m = m0 + mm;
                xs[mm][j] = (m < a.M && j < n) ? xrow[m * mstride + j] : make_float2(0.f, 0.f);
            }
            __syncthreads();
#pragma unroll 2
            for (int mm = 0; mm < AM; ++mm) {
                double2 xr[NBK], xc[NBK];
#pragma unroll
                for (int P = 0; P < NBK; ++P) {
                    const float2 u = xs[mm][32 * P + tr], v = xs[mm][32 * P + tc];
                    xr[P] = make_double2(u.x, u.y);
                    xc[P] = make_double2(v.x, v.y);
                }
#pragma unroll
                for (int P = 0; P < NBK; ++P)
#pragma unroll
                    for (int Q = 0; Q <= P; ++Q) {
                        // A[i][j] += x_i conj(x_j)
                        double2& t = A[blk(P, Q)];
                        t.x = fma(xr[P].x, xc[Q].x, fma(xr[P].y, xc[Q].y, t.x));
                        t.y = fma(xr[P].y, xc[Q].x, fma(-xr[P].x, xc[Q].y, t.y));
                    }
            }
            __syncthreads();
        }
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            A[e].x *= invM;
            A[e].y *= invM;
        }
        if (a.r_out) {
            double2* R = a.r_out + mat * n * n;
#pragma unroll
            for (int P = 0; P < NBK; ++P)
#pragma unroll
                for (int Q = 0; Q <= P; ++Q) {
                    const int i = 32 * P + tr, j = 32 * Q + tc;
                    if (i >= n || j >= n) continue;
                    const double2 v = A[blk(P, Q)];
                    R[(long long)i * n + j] = v;
                    if (P > Q) R[(long long)j * n + i] = make_double2(v.x, -v.y);
                }
        }
    }
    if (!a.want_w) return;

    // The rank-1 form of the sweep below subtracts the constants 1 (w = c - e_k)
    // and 2 at the pivot, which is exact only for entries of order one: with
    // R ~ 1e10 the pivot updates cancel to noise.  The sweep therefore works
    // on A / alpha, alpha a power of two near the largest diagonal entry of
    // R + lam I (exact scaling): W = I - lam A^-1 = I - (lam / alpha)
    // (A / alpha)^-1, and A^-1 = (A / alpha)^-1 / alpha.
    double* red = reinterpret_cast<double*>(&cb[0][0]);   // 16 wave maxima
    {
        double dm = 0.0;
#pragma unroll
        for (int P = 0; P < NBK; ++P)
            if (tr == tc && 32 * P + tr < n) dm = fmax(dm, A[blk(P, P)].x);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) dm = fmax(dm, __shfl_xor(dm, m));
        if ((tid & 63) == 0) red[tid >> 6] = dm;
        __syncthreads();
        dm = red[0];
        for (int w = 1; w < 16; ++w) dm = fmax(dm, red[w]);
        __syncthreads();   // every read of red is done before cb is cleared
        const double top = dm + a.lam;
        const double alpha = (top > 0.0 && isfinite(top)) ? exp2(rint(log2(top))) : 1.0;
        const double inva = 1.0 / alpha;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            A[e].x *= inva;
            A[e].y *= inva;
        }
        lam_s = a.lam * inva;
        ainv_s = inva;
    }
    // A = R + lam I (scaled); publish pivot column 0
#pragma unroll
    for (int P = 0; P < NBK; ++P)
        if (tr == tc && 32 * P + tr < n) A[blk(P, P)].x += lam_s;
    for (int e = tid; e < 2 * NMAX; e += 1024) cb[e / NMAX][e % NMAX] = make_double2(0.0, 0.0);
    __syncthreads();
    publish_col<NBK, 0>(A, 0, tr, tc, n, cb[0]);
    __syncthreads();

    bool ok = true;
    // Pivots kp = 32 QP + t; the block index QP is unrolled
#define LMMSE_SWEEP_GROUP(QP)                                                              \
    if (ok && 32 * (QP) < n) {                                                             \
        const int tmax = min(32, n - 32 * (QP));                                           \
        for (int t = 0; t < tmax; ++t) {                                                   \
            const int kp = 32 * (QP) + t;                                                  \
            const double2* cc = cb[kp & 1];                                                \
            double2* cn = cb[(kp + 1) & 1];                                                \
            const double d = cc[kp].x;                                                     \
            if (!(d > 0.0) || !isfinite(d)) {                                              \
                if (tid == 0 && atomicCAS(a.status, 0, LMMSE_ERR_NOT_PD) == 0)             \
                    a.status[1] = (int)(mat + a.mat0);                                                \
                ok = false; /* every thread reads the same d: uniform exit */              \
                break;                                                                     \
            }                                                                              \
            const double invd = 1.0 / d;                                                   \
            double2 wr[NBK], wc[NBK];                                                      \
            _Pragma("unroll") for (int P = 0; P < NBK; ++P) {                              \
                double2 u = cc[32 * P + tr], v = cc[32 * P + tc];                          \
                if (32 * P + tr == kp) u.x -= 1.0;                                         \
                if (32 * P + tc == kp) v.x -= 1.0;                                         \
                wr[P] = make_double2(u.x * invd, u.y * invd);                              \
                wc[P] = v;                                                                 \
            }                                                                              \
            _Pragma("unroll") for (int P = 0; P < NBK; ++P)                                \
                _Pragma("unroll") for (int Q = 0; Q <= P; ++Q) {                           \
                    double2& x = A[blk(P, Q)];                                             \
                    x.x = fma(-wr[P].x, wc[Q].x, fma(-wr[P].y, wc[Q].y, x.x));             \
                    x.y = fma(-wr[P].y, wc[Q].x, fma(wr[P].x, wc[Q].y, x.y));              \
                }                                                                          \
            if (tr == t && tc == t) A[blk(QP, QP)].x -= 2.0;                               \
            if (kp + 1 < n) {                                                              \
                if (t + 1 < 32) publish_col<NBK, (QP)>(A, t + 1, tr, tc, n, cn);           \
                else if ((QP) + 1 < NBK)                                                   \
                    publish_col<NBK, ((QP) + 1 < NBK ? (QP) + 1 : (QP))>(A, 0, tr, tc, n, cn); \
            }                                                                              \
            __syncthreads();                                                               \
        }                                                                                  \
    }
    LMMSE_SWEEP_GROUP(0)
    if constexpr (NBK > 1) { LMMSE_SWEEP_GROUP(1) }
    if constexpr (NBK > 2) { LMMSE_SWEEP_GROUP(2) }
    if constexpr (NBK > 3) { LMMSE_SWEEP_GROUP(3) }
    if constexpr (NBK > 4) { LMMSE_SWEEP_GROUP(4) }
#undef LMMSE_SWEEP_GROUP
    if (!ok) return;

    // A now holds -A^-1: W[o][j] = delta(off + o, j) + lam (-A^-1)[off + o][j]
    const int off = a.offsets[b];
    const int wp = (n + 1) & ~1, w16 = (n + 15) & ~15;
#pragma unroll
    for (int P = 0; P < NBK; ++P)
#pragma unroll
        for (int Q = 0; Q <= P; ++Q) {
            const int i = 32 * P + tr, j = 32 * Q + tc;
            if (i >= n || j >= n) continue;
            const double2 v = A[blk(P, Q)];
            if (a.ainv) {
                double2* ai = a.ainv + mat * n * n;
                ai[(long long)i * n + j] = make_double2(-v.x * ainv_s, -v.y * ainv_s);
                if (P > Q) ai[(long long)j * n + i] = make_double2(-v.x * ainv_s, v.y * ainv_s);
            }
            // entry (i, j) and, off the diagonal blocks, its mirror (j, i)
#pragma unroll
            for (int side = 0; side < (P > Q ? 2 : 1); ++side) {
                const int row = side == 0 ? i : j, col = side == 0 ? j : i;
                const int o = row - off;
                if (o < 0 || o >= a.B) continue;
                const double vy = side == 0 ? v.y : -v.y;
                const double2 w = make_double2((row == col ? 1.0 : 0.0) + lam_s * v.x, lam_s * vy);
                if (a.w64) a.w64[(mat * a.B + o) * n + col] = w;
                if (a.w32) {
                    const long long wb = mat * a.B * (long long)w16;
                    a.w32[split_w_index(wb, a.B, o, col)] = make_float2((float)w.x, (float)w.y);
                    if (col == 0)   // pad columns
                        for (int c = n; c < w16; ++c) a.w32[split_w_index(wb, a.B, o, c)] = make_float2(0.f, 0.f);
                }
                if (a.whi) store_split_w(a.whi, a.wlo, mat * a.B * (long long)w16, a.B, o, col, n, w16, w,
                                         a.split_fp16);
            }
        }
}

// ---------------------------------------------------------------- apply
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct SampleApplyArgs {
    const float2* hls;
    const float2* w32;      // compact complex filters, B x Wp per window in the chunk-major
                            // order of split_w_index, Wp = Wn rounded up to 16
    const int* starts;
    float2* out;
    long long n_tiles;
    int M, K, N, B, Wn, Wp, nb, rgroups, G16, cgroups;
};

__device__ __forceinline__ float f4s(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

constexpr int pCT = 2;                   // column tiles per wave
constexpr int pThreads = 256;            // 4 waves
constexpr int pCols = 16 * pCT * 4;      // 128 antennas per workgroup
constexpr int pXP = pCols + 1;           // LS chunk row stride (16-byte slots), slot-major

// Filter chunk cc of this row group into LDS with the direct global-to-LDS
// loads: 16-byte slot s of the buffer holds W[o][16cc + 2jp .. +1] (one
// complex pair) with o = s / 8 and jp = (s % 8) ^ (o % 8), a swizzle that
// makes the 8 rows a lane group reads at one jp fall into distinct banks.
// The window's filters are chunk-major (the 16 columns of chunk cc of all B
// rows one contiguous block, whole 128-byte rows, zero past Wn).  Rows past B
// read row B - 1 and produce discarded outputs.
template <int RT>
__device__ __forceinline__ void sample_copy_w(const float2* wmat, int B, int o0, int cc,
                                              int wave, int lane, float4* wdst) {
    constexpr int NV = RT * 64;   // 8 RT rows x 8 slots
#pragma unroll
    for (int u = 0; u < (NV + pThreads - 1) / pThreads; ++u) {
        const int base = u * pThreads + wave * 64;
        if (base < NV) {
            const int sl = base + lane, ol = sl >> 3, jp = (sl & 7) ^ (ol & 7);
            const int o = min(o0 + ol, B - 1);
            const float2* src = wmat + (unsigned)((cc * B + o) * 16 + 2 * jp);   // chunk-major
            __builtin_amdgcn_global_load_lds(
                src, (__attribute__((address_space(3))) void*)(wdst + base), 16, 0, 0);
        }
    }
}

// LS values of one chunk: 128 antennas x 16 window rows, 8 per thread.
struct SampleRaw {
    float2 v[8];
};

__device__ __forceinline__ void sample_load_x(const SampleApplyArgs& a, const float2* xbase,
                                              long long xstride, int m0, int cc, int tid,
                                              SampleRaw& R) {
    const int r = tid & 15, c0 = tid >> 4, j = 16 * cc + r;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int m = m0 + c0 + 16 * u;
        R.v[u] = (j < a.Wn && m < a.M) ? xbase[m * xstride + j] : make_float2(0.f, 0.f);
    }
}

__device__ __forceinline__ void sample_store_x(const SampleRaw& R, int tid, float4* xs4) {
    float2* xs2 = reinterpret_cast<float2*>(xs4);
    const int r = tid & 15, c0 = tid >> 4;
#pragma unroll
    for (int u = 0; u < 8; ++u) xs2[2 * ((r >> 1) * pXP + c0 + 16 * u) + (r & 1)] = R.v[u];
}

// One group of 8 window rows: per row tile the filter pair is read once and
// expanded to the real embedding [[Re, -Im], [Im, Re]] in registers.
template <int RT>
__device__ __forceinline__ void sample_mfma_group(floatx4 (&acc)[RT][pCT], const float4 (&xv)[pCT],
                                                  const float4* wb, int gg, int l16, int q) {
    const int ro = l16 & 1;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int ol = 8 * rt + (l16 >> 1), jp = 4 * gg + q;
        const float4 w = wb[8 * ol + (jp ^ (ol & 7))];
        const float4 av = ro == 0 ? make_float4(w.x, -w.y, w.z, -w.w) : make_float4(w.y, w.x, w.w, w.z);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int ct = 0; ct < pCT; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(f4s(av, i), f4s(xv[ct], i),
                                                                   acc[rt][ct], 0, 0, 0);
    }
}

struct SampleCtx {
    const SampleApplyArgs& a;
    const float2* xbase;
    const float2* wmat;
    long long xstride;
    int m0, o0, nchunks, tid, wave, lane, l16, q;
};

// One chunk, as in the fixed-path kernel: LS values into LDS, next chunk's LS
// values into registers, barrier, first group's MFMAs, the second group's LS
// operands, the copy of the next filter chunk into wnext, the second group's
// MFMAs, wait, barrier.
template <int RT>
__device__ __forceinline__ void sample_step(const SampleCtx& x, int cc, float4* xs4, float4* wcur,
                                            float4* wnext, floatx4 (&acc)[RT][pCT], SampleRaw& raw) {
    sample_store_x(raw, x.tid, xs4);
    if (cc + 1 < x.nchunks) sample_load_x(x.a, x.xbase, x.xstride, x.m0, cc + 1, x.tid, raw);
    __syncthreads();
    float4 xv[pCT];
#pragma unroll
    for (int ct = 0; ct < pCT; ++ct) xv[ct] = xs4[x.q * pXP + (x.wave * pCT + ct) * 16 + x.l16];
    sample_mfma_group<RT>(acc, xv, wcur, 0, x.l16, x.q);
#pragma unroll
    for (int ct = 0; ct < pCT; ++ct) xv[ct] = xs4[(4 + x.q) * pXP + (x.wave * pCT + ct) * 16 + x.l16];
    if (cc + 1 < x.nchunks) sample_copy_w<RT>(x.wmat, x.a.B, x.o0, cc + 1, x.wave, x.lane, wnext);
    if (16 * cc + 8 < x.a.Wn) sample_mfma_group<RT>(acc, xv, wcur, 1, x.l16, x.q);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies have landed
    __syncthreads();
}

template <int RT>
__global__ __launch_bounds__(pThreads, 2) void apply_sample_kernel(SampleApplyArgs a) {
    __shared__ float4 xs4[8 * pXP];
    __shared__ float4 wA[RT * 64];
    __shared__ float4 wB[RT * 64];
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
    const SampleCtx x{a,
                      a.hls + ((s * a.M) * a.K + k) * (long long)a.N + a.starts[b],
                      a.w32 + ((sk * a.nb + b) * a.B) * (long long)a.Wp,
                      (long long)a.K * a.N,
                      cg * pCols,
                      rg * RT * 8,
                      a.G16,
                      tid,
                      wave,
                      lane,
                      lane & 15,
                      lane >> 4};
    floatx4 acc[RT][pCT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < pCT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    SampleRaw raw;
    sample_copy_w<RT>(x.wmat, a.B, x.o0, 0, wave, lane, wA);
    sample_load_x(a, x.xbase, x.xstride, x.m0, 0, tid, raw);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    for (int cc = 0; cc < x.nchunks; cc += 2) {
        sample_step<RT>(x, cc, xs4, wA, wB, acc, raw);
        if (cc + 1 < x.nchunks) sample_step<RT>(x, cc + 1, xs4, wB, wA, acc, raw);
    }
    const int l16 = x.l16, q = x.q;
#pragma unroll
    for (int ct = 0; ct < pCT; ++ct) {
        const int m = x.m0 + (wave * pCT + ct) * 16 + l16;
        if (m >= a.M) continue;
        float2* op = a.out + ((s * a.M + m) * a.K + k) * (long long)a.N + (long long)b * a.B;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int o = (((rg * RT + rt) * 16) + 4 * q) >> 1;
            const floatx4 v = acc[rt][ct];
            if (o < a.B) op[o] = make_float2(v[0], v[1]);
            if (o + 1 < a.B) op[o + 1] = make_float2(v[2], v[3]);
        }
    }
}

// ---------------------------------------------------------------- launchers
static hipError_t launch_sample_design(const Plan& p, long long nmat, SampleArgs sa, hipStream_t st) {
    if (nmat == 0) return hipSuccess;
    const dim3 grid((unsigned)nmat), block(1024);
    if (p.d.Wn <= 32)
        hipLaunchKernelGGL((sample_design_kernel<1>), grid, block, 0, st, sa);
    else if (p.d.Wn <= 64)
        hipLaunchKernelGGL((sample_design_kernel<2>), grid, block, 0, st, sa);
    else if (p.d.Wn <= 96)
        hipLaunchKernelGGL((sample_design_kernel<3>), grid, block, 0, st, sa);
    else if (p.d.Wn <= 128)
        hipLaunchKernelGGL((sample_design_kernel<4>), grid, block, 0, st, sa);
    else if (p.d.Wn <= 160)
        hipLaunchKernelGGL((sample_design_kernel<5>), grid, block, 0, st, sa);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

static SampleArgs base_args(const Plan& p, double lam) {
    SampleArgs sa{};
    sa.starts = p.d_starts;
    sa.offsets = p.d_offsets;
    sa.status = p.status;
    sa.M = p.d.M;
    sa.K = p.d.K;
    sa.N = p.d.N;
    sa.B = p.d.B;
    sa.Wn = p.d.Wn;
    sa.nb = p.nb;
    sa.lam = lam;
    return sa;
}

hipError_t launch_covariance(const Plan& p, int slots, const float2* hls, double2* r_win,
                             hipStream_t st) {
    if (p.d.Wn > kMaxSampleWindowReg)
        return launch_covariance_large(p, (long long)slots * p.d.K * p.nb, hls, r_win, st);
    SampleArgs sa = base_args(p, 0.0);
    sa.hls = hls;
    sa.r_out = r_win;
    sa.want_w = 0;
    return launch_sample_design(p, (long long)slots * p.d.K * p.nb, sa, st);
}

hipError_t launch_batched_filters(const Plan& p, long long nmat, const double2* r_win, double lam,
                                  double2* w_out, double2* ainv, hipStream_t st) {
    SampleArgs sa = base_args(p, lam);
    sa.r_in = r_win;
    sa.w64 = w_out;
    sa.ainv = ainv;
    sa.want_w = 1;
    return launch_sample_design(p, nmat, sa, st);
}

hipError_t launch_sample_inverse(const Plan& p, long long nmat, long long mat0, const float2* hls,
                                 double lam, double2* w64, double2* ainv, double2* scratch,
                                 hipStream_t st) {
    if (p.d.Wn > kMaxSampleWindowReg)
        return launch_sample_large(p, nmat, mat0, hls, lam, ainv, scratch, w64, nullptr, nullptr,
                                   nullptr, true, st);
    if (resident_design_fits(p.d.Wn))
        return launch_resident_design(p, nmat, mat0, hls, lam, ainv, w64, nullptr, nullptr, nullptr, true, st);
    SampleArgs sa = base_args(p, lam);
    sa.mat0 = mat0;
    sa.hls = hls;
    sa.w64 = w64;
    sa.ainv = ainv;
    sa.want_w = 1;
    return launch_sample_design(p, nmat, sa, st);
}

// Slots per design chunk of the workspace-resident design (wide windows):
// up to 2 GiB of window matrices at a time, at least one slot.
static int large_chunk(const lmmse_plan_desc& d, int slots) {
    if (slots <= 0) return 0;
    const long long ms = (long long)d.K * (d.N / d.B);
    const size_t per = d.Wn > kMaxSampleWindowLarge ? pushthrough_bytes(d, ms) : large_design_bytes(d, ms);
    const size_t c = per ? ((size_t)2 << 30) / per : (size_t)slots;
    return (int)std::min<size_t>(std::max<size_t>(c, 1), (size_t)slots);
}

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Compact filters of every (slot, user, block): FP32 complex values, or hi
// and lo parts of packed 16-bit pairs, B x W16 per window (W16 = Wn rounded
// up to 16) in the chunk-major order of split_w_index.
static size_t filter_area_bytes(const lmmse_plan_desc& d, long long nmat) {
    if (d.precision == LMMSE_FP32) return up256((size_t)nmat * d.B * ((d.Wn + 15) & ~15) * sizeof(float2));
    return up256(2 * (size_t)nmat * d.B * ((d.Wn + 15) & ~15) * sizeof(uint32_t));
}

size_t sample_workspace_bytes(const lmmse_plan_desc& d, int slots) {
    // H_LS, the compact filters of every (slot, user, block), and for wide
    // windows the design work area of one chunk of slots; windows wider than
    // the workspace-resident design: H_LS and the push-through work area of
    // one chunk of slots
    const size_t hls = hls_bytes(d, slots);
    if (d.Wn > kMaxSampleWindowLarge)
        return slots > 0 ? hls + pushthrough_bytes(d, (long long)large_chunk(d, slots) * d.K * (d.N / d.B))
                         : 0;
    const size_t w = filter_area_bytes(d, (long long)slots * d.K * (d.N / d.B));
    size_t big = 0;
    if (d.Wn > kMaxSampleWindowReg && slots > 0)
        big = large_design_bytes(d, (long long)large_chunk(d, slots) * d.K * (d.N / d.B));
    return hls + w + big;
}

hipError_t launch_sample_estimate(const Plan& p, int slots, const float2* hls, double lam,
                                  float2* out, void* ws, hipStream_t st, double2* keep_w64,
                                  double2* keep_ainv) {
    const long long nmat = (long long)slots * p.d.K * p.nb;
    if (nmat == 0) return hipSuccess;
    if ((keep_w64 == nullptr) != (keep_ainv == nullptr) || (keep_w64 && !resident_design_fits(p.d.Wn)))
        return hipErrorInvalidValue;
    const bool split = p.d.precision != LMMSE_FP32;
    const int wp = (p.d.Wn + 15) & ~15, wq = wp;   // W16 for both filter formats
    float2* w32 = split ? nullptr : reinterpret_cast<float2*>(ws);
    uint32_t* whi = split ? reinterpret_cast<uint32_t*>(ws) : nullptr;
    uint32_t* wlo = split ? whi + nmat * p.d.B * wq : nullptr;
    hipError_t e;
    if (p.d.Wn > kMaxSampleWindowLarge) {   // push-through form, FP32 product
        const int chunk = large_chunk(p.d, slots);
        const long long cm = (long long)chunk * p.d.K * p.nb;
        double2* amat = reinterpret_cast<double2*>(ws);
        double2* scratch = amat + cm * p.d.M * p.d.M;
        const long long per_slot = (long long)p.d.M * p.d.K * p.d.N;
        for (int s0 = 0; s0 < slots; s0 += chunk) {
            const int ns = std::min(chunk, slots - s0);
            e = launch_sample_pushthrough(p, (long long)ns * p.d.K * p.nb, (long long)s0 * p.d.K * p.nb,
                                          hls + s0 * per_slot, lam, amat, scratch, out + s0 * per_slot,
                                          st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (resident_design_fits(p.d.Wn)) {
        // every window of every slot in one launch: the forward keeps no
        // window matrix, so nothing bounds the launch to a chunk of slots
        e = launch_resident_design(p, nmat, 0, hls, lam, keep_ainv, keep_w64, w32, whi, wlo,
                                   keep_ainv != nullptr, st);
        if (e != hipSuccess) return e;
    } else if (p.d.Wn > kMaxSampleWindowReg) {
        const int chunk = large_chunk(p.d, slots);
        const long long cm = (long long)chunk * p.d.K * p.nb;
        double2* amat = reinterpret_cast<double2*>((char*)ws + filter_area_bytes(p.d, nmat));
        double2* scratch = amat + cm * p.d.Wn * p.d.Wn;
        const long long per_slot = (long long)p.d.M * p.d.K * p.d.N;
        for (int s0 = 0; s0 < slots; s0 += chunk) {
            const int ns = std::min(chunk, slots - s0);
            const long long m0 = (long long)s0 * p.d.K * p.nb;
            e = launch_sample_large(p, (long long)ns * p.d.K * p.nb, m0, hls + s0 * per_slot, lam, amat,
                                    scratch, nullptr, split ? nullptr : w32 + m0 * p.d.B * wp,
                                    split ? whi + m0 * p.d.B * wq : nullptr,
                                    split ? wlo + m0 * p.d.B * wq : nullptr, false, st);
            if (e != hipSuccess) return e;
        }
    } else {
        SampleArgs sa = base_args(p, lam);
        sa.hls = hls;
        sa.w32 = w32;
        sa.whi = whi;
        sa.wlo = wlo;
        sa.split_fp16 = p.d.precision == LMMSE_FP16X3 ? 1 : 0;
        sa.want_w = 1;
        e = launch_sample_design(p, nmat, sa, st);
        if (e != hipSuccess) return e;
    }
    if (split) return launch_apply_sample_split(p, nmat, hls, whi, wlo, out, st);
    SampleApplyArgs aa{};
    aa.hls = hls;
    aa.w32 = w32;
    aa.starts = p.d_starts;
    aa.out = out;
    aa.M = p.d.M;
    aa.K = p.d.K;
    aa.N = p.d.N;
    aa.B = p.d.B;
    aa.Wn = p.d.Wn;
    aa.Wp = (p.d.Wn + 15) & ~15;
    aa.nb = p.nb;
    aa.rgroups = p.rgroups;
    aa.G16 = p.G16;
    aa.cgroups = (p.d.M + pCols - 1) / pCols;
    aa.n_tiles = nmat * aa.cgroups * p.rgroups;
    const dim3 grid((unsigned)aa.n_tiles), block(pThreads);
    switch (p.RT) {
#define LMMSE_SA(R) \
    case R: hipLaunchKernelGGL((apply_sample_kernel<R>), grid, block, 0, st, aa); break;
        LMMSE_SA(1) LMMSE_SA(2) LMMSE_SA(4) LMMSE_SA(8) LMMSE_SA(9) LMMSE_SA(13) LMMSE_SA(15)
        LMMSE_SA(17)
#undef LMMSE_SA
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lmmse
