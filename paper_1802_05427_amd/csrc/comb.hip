// Comb-pilot 3W / 12W LMMSE estimators (Sec. IV-B, Tables I-II, the 3W
// weights W(1..3) and P, zero-order hold of Sec. IV-C).
//
// Pilots: UE k (0-based) owns the comb tones k, k + S, k + 2S, ... (S = the
// comb spacing, N / S tones) of one pilot OFDM symbol; its LS values there
// are Y / X (eq. 9).  Groups are numbered by tone: group b's window is the
// `win` consecutive tones starting at wst_b = clamp(b - (win-1)/2, 0,
// N/S - win) (3 for 3W, 12 for 12W); its outputs are
//   3W:  the subcarriers k + S b + j S/3, j = 0, 1, 2 (those below N),
//   12W: the S subcarriers S b .. S b + S - 1,
// and W_b = R_OI (R_II + lam I)^-1 with R[a][c] = r(a - c) (eq. 13 / 17; P
// of the 3W weights read as the inverse), lam = sigma2 (one unit-modulus
// pilot symbol per LS value).  W_b depends only on the offset of b in its
// window, cls = b - wst_b (and, for 12W, on k), so each UE has `win`
// filter classes.  3W fills every subcarrier without an estimate from the
// latest estimate below it (the first estimate below the first one).
// The interpolated-LS baselines use the same LS staging: the held LS, the
// linear interpolation between a UE's tones, the 3-fold form (linear at
// the 3W output positions, then held), the quadratic through the tones
// before, at and after each interval, and the natural cubic spline.
#include <algorithm>
#include <cmath>
#include <new>

#include "internal.h"

namespace lmmse {

constexpr int kCombWinMax = 12;
constexpr int kCombOutMax = 16;
constexpr int kCombTonesMax = 4096;         // LS staging in LDS
constexpr int kCombSplineTonesMax = 2048;   // LS + second derivatives + pivots in LDS
constexpr int kCombLdsBytes = 64 * 1024;          // dynamic LDS of one apply workgroup

struct CombPlan {
    lmmse_comb_desc d{};
    int ntones = 0, win = 0, nout = 0;
    double2* w64 = nullptr;   // [K][win][nout][win]
    float2* w32 = nullptr;    // same layout
    int* status = nullptr;    // [2]
};

// r(d) of the fixed designs for a signed subcarrier difference (r(-d) =
// conj(r(d))): eq. 16 with N_fft, or the discrete exponential tap sum.
__device__ double2 comb_r(int d, int rsource, double L, double tau, int taps, int N_fft) {
    if (rsource == LMMSE_R_UNIFORM) {
        if (d == 0) return make_double2(1.0, 0.0);
        const double a = 2.0 * M_PI * L * (double)d / (double)N_fft;
        const double sh = sin(0.5 * a);
        return make_double2(sin(a) / a, -2.0 * sh * sh / a);
    }
    double S = 0.0, rx = 0.0, ry = 0.0;
    for (int l = 0; l < taps; ++l) S += exp(-(double)l / tau);
    for (int l = 0; l < taps; ++l) {
        const double p = exp(-(double)l / tau) / S;
        const long long m = (((long long)l * d) % N_fft + N_fft) % N_fft;
        double sn, cs;
        sincospi(2.0 * (double)m / (double)N_fft, &sn, &cs);
        rx += p * cs;
        ry -= p * sn;
    }
    return make_double2(rx, ry);
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One filter class (UE k = blockIdx.y, class cls = blockIdx.x) in FP64.
__global__ __launch_bounds__(256) void comb_design_kernel(lmmse_comb_desc d, int win, int nout,
                                                          double2* w64, float2* w32, int* status) {
    __shared__ double2 A[kCombWinMax][kCombWinMax];
    __shared__ double2 Ro[kCombOutMax][kCombWinMax];
    __shared__ int ok;
    const int cls = blockIdx.x, k = blockIdx.y, tid = threadIdx.x, S = d.comb;
    const double lam = d.sigma2;
    for (int e = tid; e < win * win; e += 256) {
        const int i = e / win, j = e - i * win;
        double2 v = comb_r(S * (i - j), d.rsource, d.L, d.tau_rms, d.taps, d.N_fft);
        if (i == j) v.x += lam;
        A[i][j] = v;
    }
    for (int e = tid; e < nout * win; e += 256) {
        const int o = e / win, j = e - o * win;
        // output o minus the window's first tone
        const int off = d.kind == LMMSE_COMB_12W ? S * cls + o - k : S * cls + o * (S / 3);
        Ro[o][j] = comb_r(off - S * j, d.rsource, d.L, d.tau_rms, d.taps, d.N_fft);
    }
    __syncthreads();
    if (tid == 0) {
        // in-place Gauss-Jordan inverse of the Hermitian positive definite A
        ok = 1;
        for (int p = 0; p < win && ok; ++p) {
            const double piv = A[p][p].x;
            if (!(piv > 0.0) || !isfinite(piv)) {
                ok = 0;
                break;
            }
            const double inv = 1.0 / piv;
            for (int j = 0; j < win; ++j) A[p][j] = make_double2(A[p][j].x * inv, A[p][j].y * inv);
            A[p][p] = make_double2(inv, 0.0);
            for (int i = 0; i < win; ++i) {
                if (i == p) continue;
                const double2 f = A[i][p];
                A[i][p] = make_double2(0.0, 0.0);
                for (int j = 0; j < win; ++j) {
                    const double2 t = zmul(f, A[p][j]);
                    A[i][j] = make_double2(A[i][j].x - t.x, A[i][j].y - t.y);
                }
            }
        }
        if (!ok && atomicCAS(status, 0, LMMSE_ERR_NOT_PD) == 0) status[1] = k * win + cls;
    }
    __syncthreads();
    if (!ok) return;
    const size_t base = ((size_t)k * win + cls) * nout * win;
    for (int e = tid; e < nout * win; e += 256) {
        const int o = e / win, j = e - o * win;
        double2 s = make_double2(0.0, 0.0);
        for (int i = 0; i < win; ++i) {
            const double2 t = zmul(Ro[o][i], A[i][j]);
            s.x += t.x;
            s.y += t.y;
        }
        w64[base + e] = s;
        w32[base + e] = make_float2((float)s.x, (float)s.y);
    }
}

constexpr int kCombCols = 8;   // columns per workgroup (filter classes loaded once)
constexpr int kXcds = 8;       // XCDs of the chip
// one staged column always fits beside the largest filter set (12W, S = 16)
static_assert(kCombTonesMax * 8 + kCombWinMax * kCombOutMax * kCombWinMax * 8 <= kCombLdsBytes &&
                  kCombSplineTonesMax * (2 * 8 + 4) + 8 <= kCombLdsBytes,
              "one column must fit the staging area");

// One UE k and kCombCols columns (c = slot * M + antenna) per workgroup,
// numbered so that the K workgroups of a column group run on one XCD
// (workgroups are dealt to the 8 XCDs in turn): g = 8 (K q + k) + x serves
// column group 8 q + x, and the K reads of the same pilot-symbol rows meet
// in that XCD's L2.  Per workgroup: the UE's filter classes into LDS once, then the comb LS values
// of `cs` columns at a time into LDS and one output subcarrier per thread
// (consecutive threads write consecutive subcarriers), each thread working
// out its subcarrier's filter row or interpolation weights once for the
// staged columns.  Subcarrier p belongs to group
// b = (p - k) / S (12W: p / S) and takes output j of it: 12W j = p mod S;
// 3W the latest of the group's outputs at or below p (j = 0 below the first
// tone: the hold).
//
// The spline kind first solves, per column, for the second derivatives M
// at the UE's tones (per unit tone spacing): M_0 = M_{n-1} = 0 and
//   M_{i-1} + 4 M_i + M_{i+1} = 6 (v_{i-1} - 2 v_i + v_{i+1}),  0 < i < n-1,
// by forward elimination and back substitution, then evaluates every
// subcarrier in parallel.  The pivots of the constant matrix are computed
// once per workgroup; the solves of the staged columns run side by side,
// one thread each.  KIND is the lmmse_comb_kind, fixed per instantiation.
template <int KIND>
__global__ __launch_bounds__(256) void comb_apply_kernel(lmmse_comb_desc d, int win, int nout,
                                                         int ntones, int cs, long long ncols,
                                                         const float2* y, const float2* pilots,
                                                         const float2* w32, float2* out) {
    extern __shared__ float2 sm[];
    float2* wc = sm;                            // [win][win][nout]: class, tap, output
    float2* ls = sm + win * nout * win;         // [cs][ntones]
    float2* msd = ls + cs * ntones;             // spline: [cs][ntones] second derivatives
    float* piv = (float*)(msd + cs * ntones);   // spline: [ntones] inverse pivots
    const int tid = threadIdx.x, S = d.comb, N = d.N;
    const int xcd = (int)(blockIdx.x % kXcds), r = (int)(blockIdx.x / kXcds), k = r % d.K;
    const long long grp = (long long)(r / d.K) * kXcds + xcd;
    if (grp * kCombCols >= ncols) return;   // whole workgroup: padding of the last XCD round
    constexpr bool spline = KIND == LMMSE_COMB_LS_SPLINE;
    constexpr int kWin = KIND == LMMSE_COMB_12W ? 12 : 3;   // filter kinds: equals win
    const int nw = win * nout * win;
    for (int e = tid; e < nw; e += 256) {   // from [class][output][tap]
        const int cls = e / (nout * win), r = e - cls * nout * win, o = r / win, i = r - o * win;
        wc[(cls * win + i) * nout + o] = w32[(size_t)k * nw + e];
    }
    if (spline && tid == 0) {
        // elimination of tridiag(1, 4, 1): pivot_1 = 4, pivot_i = 4 - 1 / pivot_{i-1}
        float c = 0.f;
        for (int i = 1; i < ntones - 1; ++i) {
            c = 1.0f / (4.0f - c);
            piv[i] = c;
        }
    }
    const long long c0 = grp * kCombCols;
    for (int g0 = 0; g0 < kCombCols; g0 += cs) {
        const long long cg = c0 + g0;
        if (cg >= ncols) break;   // uniform
        const int ng = (int)min((long long)min(cs, kCombCols - g0), ncols - cg);
        for (int e = tid; e < ng * ntones; e += 256) {
            const int q = e / ntones, i = e - q * ntones, t = k + S * i;
            const float2 v = y[(cg + q) * N + t], x = pilots[t];
            const float inv = 1.0f / (x.x * x.x + x.y * x.y);
            // eq. 9: Y / X = Y conj(X) / |X|^2
            ls[e] = make_float2((v.x * x.x + v.y * x.y) * inv, (v.y * x.x - v.x * x.y) * inv);
        }
        __syncthreads();
        if constexpr (spline) {
            if (tid < ng) {
                const float2* lq = ls + tid * ntones;
                float2* mq = msd + tid * ntones;
                float2 prev = make_float2(0.f, 0.f);
#pragma unroll 4
                for (int i = 1; i < ntones - 1; ++i) {
                    const float2 a = lq[i - 1], b = lq[i], e = lq[i + 1];
                    const float rx = 6.f * (a.x - 2.f * b.x + e.x), ry = 6.f * (a.y - 2.f * b.y + e.y);
                    prev = make_float2((rx - prev.x) * piv[i], (ry - prev.y) * piv[i]);
                    mq[i] = prev;
                }
                float2 next = make_float2(0.f, 0.f);
                mq[ntones - 1] = next;
#pragma unroll 4
                for (int i = ntones - 2; i >= 1; --i) {
                    const float2 v = mq[i];
                    next = make_float2(v.x - piv[i] * next.x, v.y - piv[i] * next.y);
                    mq[i] = next;
                }
                mq[0] = make_float2(0.f, 0.f);
            }
            __syncthreads();
        }
        // 12W: two neighbouring subcarriers per thread (one window read for
        // both when they share a group, as they do for even S; one 16-byte
        // store when N is even)
        if constexpr (KIND == LMMSE_COMB_12W) {
            for (int p0 = 2 * tid; p0 < N; p0 += 512) {
                const bool two = p0 + 1 < N;
                const int p1 = two ? p0 + 1 : p0;
                const int b0 = p0 / S, j0 = p0 - b0 * S, b1 = p1 / S, j1 = p1 - b1 * S;
                const int w0 = min(max(b0 - (kWin - 1) / 2, 0), ntones - kWin);
                const int w1 = min(max(b1 - (kWin - 1) / 2, 0), ntones - kWin);
                const float2* Wa = wc + (b0 - w0) * kWin * nout + j0;
                const float2* Wb = wc + (b1 - w1) * kWin * nout + j1;
                float2 wa[kWin], wb[kWin];
#pragma unroll
                for (int i = 0; i < kWin; ++i) {
                    wa[i] = Wa[i * nout];
                    wb[i] = Wb[i * nout];
                }
                const long long ob = ((cg * d.K + k) * (long long)N) + p0, ostep = (long long)d.K * N;
                for (int cq = 0; cq < ng; ++cq) {
                    const float2* lv = ls + cq * ntones;
                    float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
                    if (w0 == w1) {
#pragma unroll
                        for (int i = 0; i < kWin; ++i) {
                            const float2 x = lv[w0 + i];
                            a0.x += wa[i].x * x.x - wa[i].y * x.y;
                            a0.y += wa[i].x * x.y + wa[i].y * x.x;
                            a1.x += wb[i].x * x.x - wb[i].y * x.y;
                            a1.y += wb[i].x * x.y + wb[i].y * x.x;
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < kWin; ++i) {
                            const float2 x = lv[w0 + i], z = lv[w1 + i];
                            a0.x += wa[i].x * x.x - wa[i].y * x.y;
                            a0.y += wa[i].x * x.y + wa[i].y * x.x;
                            a1.x += wb[i].x * z.x - wb[i].y * z.y;
                            a1.y += wb[i].x * z.y + wb[i].y * z.x;
                        }
                    }
                    float2* o = out + ob + cq * ostep;
                    if (two && (N & 1) == 0) {
                        *reinterpret_cast<float4*>(o) = make_float4(a0.x, a0.y, a1.x, a1.y);
                    } else {
                        o[0] = a0;
                        if (two) o[1] = a1;
                    }
                }
            }
        } else {
        // per subcarrier: its filter row (3W) or interpolation weights, then
        // the same combination of LS values in every staged column
        for (int p = tid; p < N; p += 256) {
            const long long obase = ((cg * d.K + k) * (long long)N) + p;   // column cg
            const long long ostep = (long long)d.K * N;                    // next column
            if constexpr (KIND == LMMSE_COMB_3W) {
                int b, j;
                if (p < k) {
                    b = 0;
                    j = 0;
                } else {
                    b = min((p - k) / S, ntones - 1);
                    j = min((p - k - S * b) / (S / 3), 2);
                }
                const int wst = min(max(b - (kWin - 1) / 2, 0), ntones - kWin);
                const float2* W = wc + (b - wst) * kWin * nout + j;
                float2 wr[kWin];
#pragma unroll
                for (int i = 0; i < kWin; ++i) wr[i] = W[i * nout];
                for (int cq = 0; cq < ng; ++cq) {
                    const float2* lv = ls + cq * ntones + wst;
                    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
                    for (int i = 0; i < kWin; ++i) {
                        const float2 x = lv[i];
                        acc.x += wr[i].x * x.x - wr[i].y * x.y;
                        acc.y += wr[i].x * x.y + wr[i].y * x.x;
                    }
                    out[obase + cq * ostep] = acc;
                }
            } else if constexpr (KIND == LMMSE_COMB_LS_HOLD) {
                const int idx = p < k ? 0 : min((p - k) / S, ntones - 1);
                for (int cq = 0; cq < ng; ++cq) out[obase + cq * ostep] = ls[cq * ntones + idx];
            } else if constexpr (KIND == LMMSE_COMB_LS_LINEAR || KIND == LMMSE_COMB_LS_LINEAR3) {
                // linear interpolation between the UE's tones, at p itself
                // or (3-fold) at the 3W output position that p holds
                int qp = p;
                if constexpr (KIND == LMMSE_COMB_LS_LINEAR3) {
                    if (p >= k) {
                        const int b = min((p - k) / S, ntones - 1);
                        qp = k + S * b + min((p - k - S * b) / (S / 3), 2) * (S / 3);
                    }
                }
                int i0;
                float w0, w1;
                if (qp <= k) {
                    i0 = 0, w0 = 1.f, w1 = 0.f;
                } else if (qp >= k + S * (ntones - 1)) {
                    i0 = ntones - 2, w0 = 0.f, w1 = 1.f;
                } else {
                    i0 = (qp - k) / S;
                    w1 = (float)(qp - k - S * i0) / (float)S;
                    w0 = 1.f - w1;
                }
                for (int cq = 0; cq < ng; ++cq) {
                    const float2 v0 = ls[cq * ntones + i0], v1 = ls[cq * ntones + i0 + 1];
                    out[obase + cq * ostep] = make_float2(w0 * v0.x + w1 * v1.x, w0 * v0.y + w1 * v1.y);
                }
            } else if constexpr (KIND == LMMSE_COMB_LS_QUADRATIC) {
                // Lagrange quadratic through tones m, m+1, m+2 at x tone spacings past m
                int m;
                float l0, l1, l2;
                if (p <= k) {
                    m = 0, l0 = 1.f, l1 = 0.f, l2 = 0.f;
                } else if (p >= k + S * (ntones - 1)) {
                    m = ntones - 3, l0 = 0.f, l1 = 0.f, l2 = 1.f;
                } else {
                    m = min(max((p - k) / S - 1, 0), ntones - 3);
                    const float x = (float)(p - k - S * m) / (float)S;
                    l0 = 0.5f * (x - 1.f) * (x - 2.f), l1 = -x * (x - 2.f), l2 = 0.5f * x * (x - 1.f);
                }
                for (int cq = 0; cq < ng; ++cq) {
                    const float2* lv = ls + cq * ntones + m;
                    const float2 v0 = lv[0], v1 = lv[1], v2 = lv[2];
                    out[obase + cq * ostep] =
                        make_float2(l0 * v0.x + l1 * v1.x + l2 * v2.x, l0 * v0.y + l1 * v1.y + l2 * v2.y);
                }
            } else {   // spline
                int i0;
                float t, u, ca, cb;
                if (p <= k) {
                    i0 = 0, t = 1.f, u = 0.f;
                } else if (p >= k + S * (ntones - 1)) {
                    i0 = ntones - 2, t = 0.f, u = 1.f;
                } else {
                    i0 = (p - k) / S;
                    u = (float)(p - k - S * i0) / (float)S;
                    t = 1.f - u;
                }
                ca = (t * t * t - t) * (1.f / 6.f);   // zero at the tones
                cb = (u * u * u - u) * (1.f / 6.f);
                for (int cq = 0; cq < ng; ++cq) {
                    const float2 v0 = ls[cq * ntones + i0], v1 = ls[cq * ntones + i0 + 1];
                    const float2 m0 = msd[cq * ntones + i0], m1 = msd[cq * ntones + i0 + 1];
                    out[obase + cq * ostep] = make_float2(t * v0.x + u * v1.x + ca * m0.x + cb * m1.x,
                                                          t * v0.y + u * v1.y + ca * m0.y + cb * m1.y);
                }
            }
        }
        }
        __syncthreads();
    }
}

}  // namespace lmmse

using lmmse::CombPlan;

struct lmmse_comb {
    CombPlan p;
};

namespace {
int comb_validate(const lmmse_comb_desc* d) {
    if (!d) return LMMSE_ERR_INVALID_ARG;
    if (d->M < 1 || d->K < 1 || d->comb < 1 || d->N < 1 || d->N_fft < 1 || d->max_slots < 1)
        return LMMSE_ERR_INVALID_ARG;
    if (d->kind < LMMSE_COMB_3W || d->kind > LMMSE_COMB_LS_SPLINE) return LMMSE_ERR_INVALID_ARG;
    if (d->rsource != LMMSE_R_UNIFORM && d->rsource != LMMSE_R_EXPONENTIAL) return LMMSE_ERR_INVALID_ARG;
    if (!(d->sigma2 > 0.0) || !std::isfinite(d->sigma2)) return LMMSE_ERR_INVALID_ARG;
    if (d->rsource == LMMSE_R_UNIFORM && (!(d->L > 0.0) || !std::isfinite(d->L))) return LMMSE_ERR_INVALID_ARG;
    if (d->rsource == LMMSE_R_EXPONENTIAL &&
        (!(d->tau_rms > 0.0) || !std::isfinite(d->tau_rms) || d->taps < 1 || d->taps > d->N_fft))
        return LMMSE_ERR_INVALID_ARG;
    if (d->N > d->N_fft || d->K > d->comb || d->N % d->comb != 0) return LMMSE_ERR_UNSUPPORTED;
    const bool three = d->kind == LMMSE_COMB_3W || d->kind == LMMSE_COMB_LS_LINEAR3;
    if (three && d->comb % 3 != 0) return LMMSE_ERR_UNSUPPORTED;
    if (d->kind == LMMSE_COMB_12W && d->comb > lmmse::kCombOutMax) return LMMSE_ERR_UNSUPPORTED;
    const int win = d->kind == LMMSE_COMB_12W ? 12
                    : (d->kind == LMMSE_COMB_3W || d->kind == LMMSE_COMB_LS_QUADRATIC ||
                       d->kind == LMMSE_COMB_LS_SPLINE) ? 3 : 2;
    if (d->N / d->comb < win) return LMMSE_ERR_UNSUPPORTED;
    if (d->N / d->comb > (d->kind == LMMSE_COMB_LS_SPLINE ? lmmse::kCombSplineTonesMax
                                                          : lmmse::kCombTonesMax))
        return LMMSE_ERR_UNSUPPORTED;
    return LMMSE_OK;
}
}  // namespace

extern "C" {

int lmmse_comb_validate(const lmmse_comb_desc* d) { return comb_validate(d); }

int lmmse_comb_create(const lmmse_comb_desc* desc, lmmse_comb_t* out) {
    if (!out) return LMMSE_ERR_INVALID_ARG;
    const int v = comb_validate(desc);
    if (v != LMMSE_OK) return v;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return LMMSE_ERR_NO_DEVICE;
    lmmse_comb* c = new (std::nothrow) lmmse_comb();
    if (!c) return LMMSE_ERR_HIP;
    CombPlan& p = c->p;
    p.d = *desc;
    p.ntones = desc->N / desc->comb;
    const bool filt = desc->kind == LMMSE_COMB_3W || desc->kind == LMMSE_COMB_12W;
    p.win = desc->kind == LMMSE_COMB_12W ? 12 : (desc->kind == LMMSE_COMB_3W ? 3 : 1);
    p.nout = desc->kind == LMMSE_COMB_12W ? desc->comb : (desc->kind == LMMSE_COMB_3W ? 3 : 1);
    const size_t nw = (size_t)desc->K * p.win * p.nout * p.win;
    if (hipMalloc(&p.w64, nw * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p.w32, nw * sizeof(float2)) != hipSuccess ||
        hipMalloc(&p.status, 2 * sizeof(int)) != hipSuccess || hipMemset(p.status, 0, 2 * sizeof(int)) != hipSuccess) {
        lmmse_comb_destroy(c);
        return LMMSE_ERR_HIP;
    }
    if (filt)
        hipLaunchKernelGGL(lmmse::comb_design_kernel, dim3(p.win, desc->K), dim3(256), 0, 0, p.d,
                           p.win, p.nout, p.w64, p.w32, p.status);
    else if (hipMemset(p.w64, 0, nw * sizeof(double2)) != hipSuccess ||
             hipMemset(p.w32, 0, nw * sizeof(float2)) != hipSuccess) {
        lmmse_comb_destroy(c);
        return LMMSE_ERR_HIP;
    }
    int st[2] = {0, 0};
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(st, p.status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) {
        lmmse_comb_destroy(c);
        return LMMSE_ERR_HIP;
    }
    if (st[0]) {
        lmmse_comb_destroy(c);
        return st[0];
    }
    *out = c;
    return LMMSE_OK;
}

int lmmse_comb_destroy(lmmse_comb_t c) {
    if (!c) return LMMSE_ERR_INVALID_ARG;
    (void)hipDeviceSynchronize();
    if (c->p.w64) (void)hipFree(c->p.w64);
    if (c->p.w32) (void)hipFree(c->p.w32);
    if (c->p.status) (void)hipFree(c->p.status);
    delete c;
    return LMMSE_OK;
}

int lmmse_comb_get_filters(lmmse_comb_t c, void* w_out, void* stream) {
    if (!c || !w_out) return LMMSE_ERR_INVALID_ARG;
    const CombPlan& p = c->p;
    const size_t nw = (size_t)p.d.K * p.win * p.nout * p.win;
    if (hipMemcpyAsync(w_out, p.w64, nw * sizeof(double2), hipMemcpyDeviceToDevice,
                       (hipStream_t)stream) != hipSuccess)
        return LMMSE_ERR_HIP;
    return LMMSE_OK;
}

int lmmse_comb_estimate(lmmse_comb_t c, int slots, const void* y, const void* pilots, void* h_hat,
                        void* stream) {
    if (!c || slots < 0 || slots > c->p.d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (slots == 0) return LMMSE_OK;
    if (!y || !pilots || !h_hat) return LMMSE_ERR_INVALID_ARG;
    const CombPlan& p = c->p;
    const long long ncols = (long long)slots * p.d.M;
    const bool spline = p.d.kind == LMMSE_COMB_LS_SPLINE;
    // as many columns staged together as fit, beside the filter classes (and
    // the spline's pivots), in kCombLdsBytes of LS values (and, for the
    // spline, second derivatives); one column always fits
    const int per_col = p.ntones * (spline ? 2 : 1) * (int)sizeof(float2);
    const int fixed = p.win * p.nout * p.win * (int)sizeof(float2) + (spline ? p.ntones * (int)sizeof(float) : 0);
    const int cs = std::max(1, std::min(lmmse::kCombCols, (lmmse::kCombLdsBytes - fixed) / per_col));
    size_t shm = ((size_t)cs * p.ntones + (size_t)p.win * p.nout * p.win) * sizeof(float2);
    if (spline) shm += (size_t)cs * p.ntones * sizeof(float2) + (size_t)p.ntones * sizeof(float);
    const long long ngrp = (ncols + lmmse::kCombCols - 1) / lmmse::kCombCols;
    const long long nwg = (ngrp + lmmse::kXcds - 1) / lmmse::kXcds * lmmse::kXcds * p.d.K;
    if (nwg > 0x7fffffffLL) return LMMSE_ERR_UNSUPPORTED;
    decltype(&lmmse::comb_apply_kernel<LMMSE_COMB_3W>) kern = nullptr;
    switch (p.d.kind) {
        case LMMSE_COMB_3W: kern = lmmse::comb_apply_kernel<LMMSE_COMB_3W>; break;
        case LMMSE_COMB_12W: kern = lmmse::comb_apply_kernel<LMMSE_COMB_12W>; break;
        case LMMSE_COMB_LS_HOLD: kern = lmmse::comb_apply_kernel<LMMSE_COMB_LS_HOLD>; break;
        case LMMSE_COMB_LS_LINEAR: kern = lmmse::comb_apply_kernel<LMMSE_COMB_LS_LINEAR>; break;
        case LMMSE_COMB_LS_LINEAR3: kern = lmmse::comb_apply_kernel<LMMSE_COMB_LS_LINEAR3>; break;
        case LMMSE_COMB_LS_QUADRATIC: kern = lmmse::comb_apply_kernel<LMMSE_COMB_LS_QUADRATIC>; break;
        case LMMSE_COMB_LS_SPLINE: kern = lmmse::comb_apply_kernel<LMMSE_COMB_LS_SPLINE>; break;
        default: return LMMSE_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(256), shm, (hipStream_t)stream, p.d, p.win,
                       p.nout, p.ntones, cs, ncols, (const float2*)y, (const float2*)pilots, p.w32,
                       (float2*)h_hat);
    return hipGetLastError() == hipSuccess ? LMMSE_OK : LMMSE_ERR_HIP;
}

}  // extern "C"
