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
// linear interpolation between a UE's tones, and the 3-fold form (linear at
// the 3W output positions, then held).
#include <algorithm>
#include <cmath>
#include <new>

#include "internal.h"

namespace lmmse {

constexpr int kCombWinMax = 12;
constexpr int kCombOutMax = 16;

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

// UE k = blockIdx.y and kCombCols columns (c = slot * M + antenna) per
// workgroup: the UE's filter classes into LDS once, then per column its comb
// LS values into LDS and one output subcarrier per thread (consecutive
// threads write consecutive subcarriers).  Subcarrier p belongs to group
// b = (p - k) / S (12W: p / S) and takes output j of it: 12W j = p mod S;
// 3W the latest of the group's outputs at or below p (j = 0 below the first
// tone: the hold).
__global__ __launch_bounds__(256) void comb_apply_kernel(lmmse_comb_desc d, int win, int nout,
                                                         int ntones, long long ncols, const float2* y,
                                                         const float2* pilots, const float2* w32,
                                                         float2* out) {
    extern __shared__ float2 sm[];
    float2* wc = sm;                        // [win][nout][win]
    float2* ls = sm + win * nout * win;     // [ntones]
    const int k = blockIdx.y, tid = threadIdx.x, S = d.comb, N = d.N;
    const int nw = win * nout * win;
    for (int e = tid; e < nw; e += 256) wc[e] = w32[(size_t)k * nw + e];
    const long long c0 = (long long)blockIdx.x * kCombCols;
    for (int cc = 0; cc < kCombCols; ++cc) {
        const long long c = c0 + cc;
        if (c >= ncols) break;   // uniform
        const float2* yc = y + c * N;
        for (int i = tid; i < ntones; i += 256) {
            const int t = k + S * i;
            const float2 v = yc[t], x = pilots[t];
            const float inv = 1.0f / (x.x * x.x + x.y * x.y);
            // eq. 9: Y / X = Y conj(X) / |X|^2
            ls[i] = make_float2((v.x * x.x + v.y * x.y) * inv, (v.y * x.x - v.x * x.y) * inv);
        }
        __syncthreads();
        float2* oc = out + (c * d.K + k) * (long long)N;
        for (int p = tid; p < N; p += 256) {
            int b, j;
            if (d.kind == LMMSE_COMB_12W) {
                b = p / S;
                j = p - b * S;
            } else if (d.kind == LMMSE_COMB_LS_HOLD || d.kind == LMMSE_COMB_LS_LINEAR) {
                b = 0;
                j = 0;
            } else if (p < k) {
                b = 0;
                j = 0;
            } else {
                b = min((p - k) / S, ntones - 1);
                j = min((p - k - S * b) / (S / 3), 2);
            }
            float2 acc = make_float2(0.f, 0.f);
            if (d.kind == LMMSE_COMB_3W || d.kind == LMMSE_COMB_12W) {
                const int wst = min(max(b - (win - 1) / 2, 0), ntones - win);
                const float2* W = wc + ((b - wst) * nout + j) * win;
                for (int i = 0; i < win; ++i) {
                    const float2 w = W[i], x = ls[wst + i];
                    acc.x += w.x * x.x - w.y * x.y;
                    acc.y += w.x * x.y + w.y * x.x;
                }
            } else if (d.kind == LMMSE_COMB_LS_HOLD) {
                acc = ls[p < k ? 0 : min((p - k) / S, ntones - 1)];
            } else {
                // linear interpolation between the UE's tones, at p itself
                // or (3-fold) at the 3W output position that p holds
                const int q = d.kind == LMMSE_COMB_LS_LINEAR ? p : k + S * b + j * (S / 3);
                if (q <= k) {
                    acc = ls[0];
                } else if (q >= k + S * (ntones - 1)) {
                    acc = ls[ntones - 1];
                } else {
                    const int i0 = (q - k) / S;
                    const float f = (float)(q - k - S * i0) / (float)S;
                    acc = make_float2((1.f - f) * ls[i0].x + f * ls[i0 + 1].x,
                                      (1.f - f) * ls[i0].y + f * ls[i0 + 1].y);
                }
            }
            oc[p] = acc;
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
    if (d->kind < LMMSE_COMB_3W || d->kind > LMMSE_COMB_LS_LINEAR3) return LMMSE_ERR_INVALID_ARG;
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
    const int win = d->kind == LMMSE_COMB_12W ? 12 : (d->kind == LMMSE_COMB_3W ? 3 : 2);
    if (d->N / d->comb < win) return LMMSE_ERR_UNSUPPORTED;
    if (d->N / d->comb > 4096) return LMMSE_ERR_UNSUPPORTED;   // LS staging fits in LDS
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
    const size_t shm = ((size_t)p.ntones + (size_t)p.win * p.nout * p.win) * sizeof(float2);
    const long long nblk = (ncols + lmmse::kCombCols - 1) / lmmse::kCombCols;
    hipLaunchKernelGGL(lmmse::comb_apply_kernel, dim3((unsigned)nblk, p.d.K), dim3(256), shm,
                       (hipStream_t)stream, p.d, p.win, p.nout, p.ntones, ncols, (const float2*)y,
                       (const float2*)pilots, p.w32, (float2*)h_hat);
    return hipGetLastError() == hipSuccess ? LMMSE_OK : LMMSE_ERR_HIP;
}

}  // extern "C"
