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
// M antennas, on v_mfma_f32_16x16x4f32 with the operand layout of the fixed
// path (apply_f32.hip); the loader waves expand the compact complex W into
// its real embedding in LDS.
#include "internal.h"

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
    float2* w32;            // optional: W [mat][B][Wn]
    const int* starts;
    const int* offsets;
    int* status;
    int M, K, N, B, Wn, nb;
    double lam;
    int want_w;
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

    // A = R + lam I; publish pivot column 0
#pragma unroll
    for (int P = 0; P < NBK; ++P)
        if (tr == tc && 32 * P + tr < n) A[blk(P, P)].x += a.lam;
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
                    a.status[1] = (int)mat;                                                \
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
#pragma unroll
    for (int P = 0; P < NBK; ++P)
#pragma unroll
        for (int Q = 0; Q <= P; ++Q) {
            const int i = 32 * P + tr, j = 32 * Q + tc;
            if (i >= n || j >= n) continue;
            const double2 v = A[blk(P, Q)];
            // entry (i, j) and, off the diagonal blocks, its mirror (j, i)
#pragma unroll
            for (int side = 0; side < (P > Q ? 2 : 1); ++side) {
                const int row = side == 0 ? i : j, col = side == 0 ? j : i;
                const int o = row - off;
                if (o < 0 || o >= a.B) continue;
                const double vy = side == 0 ? v.y : -v.y;
                const double2 w = make_double2((row == col ? 1.0 : 0.0) + a.lam * v.x, a.lam * vy);
                const long long wi = (mat * a.B + o) * n + col;
                if (a.w64) a.w64[wi] = w;
                if (a.w32) a.w32[wi] = make_float2((float)w.x, (float)w.y);
            }
        }
}

// ---------------------------------------------------------------- apply
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct SampleApplyArgs {
    const float2* hls;
    const float2* w32;      // [mat][B][Wn]
    const int* starts;
    float2* out;
    long long n_tiles;
    int M, K, N, B, Wn, nb, rgroups, G8, cgroups;
};

__device__ __forceinline__ float f4s(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

constexpr int pCT = 2, pMW = 4, pLW = 2;
constexpr int pCols = 16 * pCT * pMW;    // 128 antennas per workgroup
constexpr int pXS = 18;
constexpr int pXBuf = pCols * pXS / 2;

template <int RT>
__device__ __forceinline__ void sample_stage(const SampleApplyArgs& a, int lt, int cc, int st,
                                             const float2* xbase, long long xstride, int m0,
                                             const float2* wmat, int rg, float4* ws4, float4* xs4) {
    constexpr int NL = 64 * pLW;
    // filter rows [rg*RT*16, +RT*16) of the real embedding, window rows [16cc, 16cc+16)
    for (int e = lt; e < 2 * RT * 64; e += NL) {
        const int gg = e / (RT * 64), rem = e - gg * (RT * 64);
        const int rr = rem >> 2, q = rem & 3;
        const int row = rg * RT * 16 + rr;
        const int o = row >> 1, ro = row & 1;
        const int j0 = 16 * cc + 8 * gg + 2 * q;
        float2 w0 = make_float2(0.f, 0.f), w1 = make_float2(0.f, 0.f);
        if (o < a.B) {
            if (j0 < a.Wn) w0 = wmat[(long long)o * a.Wn + j0];
            if (j0 + 1 < a.Wn) w1 = wmat[(long long)o * a.Wn + j0 + 1];
        }
        ws4[e] = ro == 0 ? make_float4(w0.x, -w0.y, w1.x, -w1.y) : make_float4(w0.y, w0.x, w1.y, w1.x);
    }
    float2* xs2 = reinterpret_cast<float2*>(xs4);
    for (int e = lt; e < pCols * 16; e += NL) {
        const int c = e >> 4, r = e & 15;
        const int j = cc * 16 + r;
        const int m = m0 + c;
        float2 v = make_float2(0.f, 0.f);
        if (j < a.Wn && m < a.M) v = xbase[m * xstride + st + j];
        xs2[c * pXS + r] = v;
    }
}

template <int RT>
__global__ __launch_bounds__(64 * (pMW + pLW)) void apply_sample_kernel(SampleApplyArgs a) {
    __shared__ float4 xs4[2 * pXBuf];
    __shared__ float4 ws4[2 * 2 * RT * 64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l16 = lane & 15, q = lane >> 4;
    long long t = blockIdx.x;
    const int rg = (int)(t % a.rgroups);
    t /= a.rgroups;
    const int cg = (int)(t % a.cgroups);
    t /= a.cgroups;
    const int b = (int)(t % a.nb);
    const long long sk = t / a.nb;
    const int k = (int)(sk % a.K);
    const long long s = sk / a.K;
    const int st = a.starts[b];
    const int m0 = cg * pCols;
    const long long xstride = (long long)a.K * a.N;
    const float2* xbase = a.hls + ((s * a.M) * a.K + k) * (long long)a.N;
    const float2* wmat = a.w32 + ((sk * a.nb + b) * a.B) * (long long)a.Wn;
    const int nchunks = (a.Wn + 15) >> 4;

    if (wave >= pMW) {
        const int lt = tid - 64 * pMW;
        sample_stage<RT>(a, lt, 0, st, xbase, xstride, m0, wmat, rg, ws4, xs4);
        __syncthreads();
        for (int cc = 0; cc < nchunks; ++cc) {
            const int nb2 = (cc + 1) & 1;
            if (cc + 1 < nchunks)
                sample_stage<RT>(a, lt, cc + 1, st, xbase, xstride, m0, wmat, rg,
                                 ws4 + nb2 * 2 * RT * 64, xs4 + nb2 * pXBuf);
            __syncthreads();
        }
        return;
    }
    floatx4 acc[RT][pCT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < pCT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    for (int cc = 0; cc < nchunks; ++cc) {
        const int buf = cc & 1;
        const float4* wb = ws4 + buf * 2 * RT * 64;
        const float4* xb = xs4 + buf * pXBuf;
#pragma unroll
        for (int gg = 0; gg < 2; ++gg) {
            float4 av[RT], xv[pCT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) av[rt] = wb[gg * RT * 64 + (rt * 16 + l16) * 4 + q];
#pragma unroll
            for (int ct = 0; ct < pCT; ++ct)
                xv[ct] = xb[((wave * pCT + ct) * 16 + l16) * (pXS / 2) + 4 * gg + q];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int ct = 0; ct < pCT; ++ct)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(f4s(av[rt], i), f4s(xv[ct], i),
                                                                           acc[rt][ct], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int ct = 0; ct < pCT; ++ct) {
        const int m = m0 + (wave * pCT + ct) * 16 + l16;
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
    SampleArgs sa = base_args(p, 0.0);
    sa.hls = hls;
    sa.r_out = r_win;
    sa.want_w = 0;
    return launch_sample_design(p, (long long)slots * p.d.K * p.nb, sa, st);
}

hipError_t launch_batched_filters(const Plan& p, int nmat, double2*, double2*, const double2* r_win,
                                  double lam, double2* w_out, hipStream_t st) {
    SampleArgs sa = base_args(p, lam);
    sa.r_in = r_win;
    sa.w64 = w_out;
    sa.want_w = 1;
    return launch_sample_design(p, nmat, sa, st);
}

size_t sample_workspace_bytes(const lmmse_plan_desc& d, int slots) {
    // H_LS, then the compact FP32 filters of every (slot, user, block)
    const size_t hls = (size_t)slots * d.M * d.K * d.N * sizeof(float2);
    const size_t w = (size_t)slots * d.K * (d.N / d.B) * d.B * d.Wn * sizeof(float2);
    return hls + w;
}

hipError_t launch_sample_estimate(const Plan& p, int slots, const float2* hls, double lam,
                                  float2* out, void* ws, hipStream_t st) {
    const long long nmat = (long long)slots * p.d.K * p.nb;
    if (nmat == 0) return hipSuccess;
    float2* w32 = reinterpret_cast<float2*>(ws);
    SampleArgs sa = base_args(p, lam);
    sa.hls = hls;
    sa.w32 = w32;
    sa.want_w = 1;
    hipError_t e = launch_sample_design(p, nmat, sa, st);
    if (e != hipSuccess) return e;
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
    aa.nb = p.nb;
    aa.rgroups = p.rgroups;
    aa.G8 = p.G8;
    aa.cgroups = (p.d.M + pCols - 1) / pCols;
    aa.n_tiles = nmat * aa.cgroups * p.rgroups;
    const dim3 grid((unsigned)aa.n_tiles), block(64 * (pMW + pLW));
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
