// Sample-covariance design for windows wider than the register-resident sweep
// of sample.hip holds (160 < Wn <= 256).  The window matrix lives in the
// workspace as FP64 [mat][Wn][Wn] (both triangles):
//
//   1. R = X X^H / M with X = h_ls[s, :, k, I_b]^T: a batched GEMM with FP64
//      accumulation of the exact products of the FP32 LS values, on the
//      lower tiles only (the upper ones are their mirror);
//   2. A = R + lam I;
//   3. the Hermitian sweep of all Wn pivots, in panels of 64 pivots K (rest
//      R): sweeping a panel at once maps
//          A_KK -> -A_KK^-1,  A_RK -> A_RK A_KK^-1,  A_KR -> A_KK^-1 A_KR,
//          A_RR -> A_RR - A_RK A_KK^-1 A_KR,
//      which equals sweeping its pivots one by one.  The panel kernel sweeps
//      the 64 x 64 diagonal block in LDS and forms F = A_RK A_KK^-1; the
//      update of A_RR is a rank-64 GEMM, A += (-1) F P^H with P the old
//      panel columns (rows of K zero in F and P, so the K rows and columns
//      are left alone).  After all panels A holds -A^-1;
//   4. W = (I - lam A^-1)[off rows] (FP64 and compact FP32 copies) and,
//      when asked for, A^-1 itself.
#include <algorithm>

#include "split.h"
#include "zgemm.h"

namespace lmmse {

constexpr int kPW = kSweepPanel;
constexpr int kPR = 16;   // window rows per staging step of the panel kernel

// A = R + lam I on the diagonal of every window.
__global__ __launch_bounds__(256) void add_diag_kernel(double2* a, int Wn, double lam) {
    double2* am = a + (long long)blockIdx.x * Wn * Wn;
    for (int i = threadIdx.x; i < Wn; i += 256) am[(long long)i * Wn + i].x += lam;
}

// Panel step over pivots [k0, k0 + kw) of every window: sweeps A_KK in LDS,
// then, 16 window rows at a time, forms F = A_RK A_KK^-1 and the GEMM
// operands F and P (old panel columns), both [mat][Wn][kPW] with zero rows in
// K and zero columns >= kw, and writes A_RK = F, A_KR = F^H and A_KK.
// Every read of a panel column happens before this thread group overwrites it:
// rows are staged, then written, one group at a time, and A_KR lies outside
// the panel columns.
__global__ __launch_bounds__(1024) void sweep_panel_kernel(double2* a, double2* f, double2* pold,
                                                           int Wn, int k0, int kw, int* status,
                                                           long long mat0) {
    __shared__ double2 D[kPW][kPW];
    __shared__ double2 Pr[kPR][kPW];
    const long long mat = blockIdx.x;
    double2* am = a + mat * Wn * Wn;
    const int tid = threadIdx.x;
    constexpr int EPT = kPW * kPW / 1024;   // entries of D per thread
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + 1024 * u, i = e / kPW, j = e - i * kPW;
        D[i][j] = (i < kw && j < kw) ? am[(long long)(k0 + i) * Wn + k0 + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int p = 0; p < kw; ++p) {
        const double d = D[p][p].x;
        if (!(d > 0.0) || !isfinite(d)) {   // the same d for every thread: uniform exit
            if (tid == 0 && atomicCAS(status, 0, LMMSE_ERR_NOT_PD) == 0)
                status[1] = (int)(mat + mat0);
            return;
        }
        const double invd = 1.0 / d;
        double2 r[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + 1024 * u, i = e / kPW, j = e - i * kPW;
            const double2 v = D[i][j], aip = D[i][p], apj = D[p][j];
            if (i == p && j == p) {
                r[u] = make_double2(-invd, 0.0);
            } else if (i == p) {
                r[u] = make_double2(apj.x * invd, apj.y * invd);
            } else if (j == p) {
                r[u] = make_double2(aip.x * invd, aip.y * invd);
            } else {
                const double px = aip.x * apj.x - aip.y * apj.y, py = aip.x * apj.y + aip.y * apj.x;
                r[u] = make_double2(v.x - px * invd, v.y - py * invd);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + 1024 * u, i = e / kPW, j = e - i * kPW;
            if (i < kw && j < kw) D[i][j] = r[u];
        }
        __syncthreads();
    }
    // D = -A_KK^-1; F = A_RK A_KK^-1 = -A_RK D, kPR rows at a time
    double2* fm = f + mat * Wn * kPW;
    double2* pm = pold + mat * Wn * kPW;
    const int ri = tid / kPW, t = tid - ri * kPW;   // this thread's (row, column) of a group
    for (int i0 = 0; i0 < Wn; i0 += kPR) {
        {
            const int i = i0 + ri;
            Pr[ri][t] = (i < Wn && t < kw) ? am[(long long)i * Wn + k0 + t] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const int i = i0 + ri;
        if (i < Wn) {
            const bool inK = i >= k0 && i < k0 + kw;
            double2 fv = make_double2(0.0, 0.0), pv = make_double2(0.0, 0.0);
            if (!inK && t < kw) {
                double sx = 0.0, sy = 0.0;
                for (int q = 0; q < kw; ++q) {
                    const double2 x = Pr[ri][q], y = D[q][t];
                    sx = fma(x.x, y.x, fma(-x.y, y.y, sx));
                    sy = fma(x.x, y.y, fma(x.y, y.x, sy));
                }
                fv = make_double2(-sx, -sy);
                pv = Pr[ri][t];
                am[(long long)i * Wn + k0 + t] = fv;
                am[(long long)(k0 + t) * Wn + i] = make_double2(fv.x, -fv.y);
            }
            fm[(long long)i * kPW + t] = fv;
            pm[(long long)i * kPW + t] = pv;
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + 1024 * u, i = e / kPW, j = e - i * kPW;
        if (i < kw && j < kw) am[(long long)(k0 + i) * Wn + k0 + j] = D[i][j];
    }
}

// W[o][j] = delta(off + o, j) + lam S[off + o][j] with S = -A^-1 as the sweep
// leaves it; optionally A^-1 = -S in place.
__global__ __launch_bounds__(256) void large_filters_kernel(double2* a, const int* offsets, int B,
                                                            int Wn, int nb, double lam, double2* w64,
                                                            float2* w32, uint32_t* whi, uint32_t* wlo,
                                                            int fp16, int negate) {
    const long long mat = blockIdx.x;
    double2* am = a + mat * Wn * Wn;
    const int off = offsets[mat % nb];
    const int wp = (Wn + 1) & ~1;
    for (int e = threadIdx.x; e < B * wp; e += 256) {
        const int o = e / wp, j = e - o * wp;
        if (j >= Wn) {
            if (w32) w32[(mat * B + o) * wp + j] = make_float2(0.f, 0.f);
            continue;
        }
        const double2 s = am[(long long)(off + o) * Wn + j];
        const double2 w = make_double2((off + o == j ? 1.0 : 0.0) + lam * s.x, lam * s.y);
        if (w64) w64[(mat * B + o) * Wn + j] = w;
        if (w32) w32[(mat * B + o) * wp + j] = make_float2((float)w.x, (float)w.y);
        if (whi) store_split_w(whi, wlo, (mat * B + o) * ((Wn + 3) & ~3), j, Wn, (Wn + 3) & ~3, w, fp16);
    }
    if (negate) {
        __syncthreads();   // every read of S above is done
        for (long long e = threadIdx.x; e < (long long)Wn * Wn; e += 256) {
            const double2 s = am[e];
            am[e] = make_double2(-s.x, -s.y);
        }
    }
}

size_t large_design_bytes(const lmmse_plan_desc& d, long long nmat) {
    const size_t per = (size_t)d.Wn * d.Wn * sizeof(double2) + 2 * (size_t)d.Wn * kPW * sizeof(double2);
    return (size_t)nmat * per;
}

hipError_t launch_sample_large(const Plan& p, long long nmat, long long mat0, const float2* hls,
                               double lam, double2* amat, double2* scratch, double2* w64,
                               float2* w32, uint32_t* whi, uint32_t* wlo, bool want_ainv,
                               hipStream_t st) {
    const lmmse_plan_desc& d = p.d;
    const int Wn = d.Wn;
    if (nmat == 0) return hipSuccess;
    if (Wn > kMaxSampleWindowLarge) return hipErrorInvalidValue;
    hipError_t e;
    // R = X X^H / M
    ZGemmArgs ga{};
    ga.K = d.K;
    ga.nb = p.nb;
    const long long ms = (long long)d.K * d.N;
    ga.A = ZView{hls, 1, ms, (long long)d.M * d.K * d.N, d.N, 1, p.d_starts, 0};
    ga.B = ZView{hls, ms, 1, (long long)d.M * d.K * d.N, d.N, 1, p.d_starts, 1};
    const long long per = (long long)Wn * Wn;
    ga.C = ZView{amat, Wn, 1, per * p.nb * d.K, per * p.nb, per, nullptr, 0};
    ga.m = Wn;
    ga.n = Wn;
    ga.kd = d.M;
    ga.alpha = 1.0 / d.M;
    ga.beta = 0;
    ga.herm = 1;
    if ((e = zgemm<float2, float2, double2>(ga, nmat, st)) != hipSuccess) return e;
    ga.herm = 0;
    hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)nmat), dim3(256), 0, st, amat, Wn, lam);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double2* f = scratch;
    double2* pold = scratch + nmat * Wn * kPW;
    const long long pp = (long long)Wn * kPW;
    for (int k0 = 0; k0 < Wn; k0 += kPW) {
        const int kw = std::min(kPW, Wn - k0);
        hipLaunchKernelGGL(sweep_panel_kernel, dim3((unsigned)nmat), dim3(1024), 0, st, amat, f, pold,
                           Wn, k0, kw, p.status, mat0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // A += (-1) F P^H over the whole window (F, P vanish on the panel's rows)
        ga.A = ZView{f, kPW, 1, pp * p.nb * d.K, pp * p.nb, pp, nullptr, 0};
        ga.B = ZView{pold, 1, kPW, pp * p.nb * d.K, pp * p.nb, pp, nullptr, 1};
        ga.C = ZView{amat, Wn, 1, per * p.nb * d.K, per * p.nb, per, nullptr, 0};
        ga.kd = kw;
        ga.alpha = -1.0;
        ga.beta = 1;
        ga.herm = 1;   // F P^H = A_RK A_KK^-1 A_RK^H is Hermitian
        if ((e = zgemm<double2, double2, double2>(ga, nmat, st)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(large_filters_kernel, dim3((unsigned)nmat), dim3(256), 0, st, amat,
                       p.d_offsets, d.B, Wn, p.nb, lam, w64, w32, whi, wlo,
                       d.precision == LMMSE_FP16X3 ? 1 : 0, want_ainv ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_covariance_large(const Plan& p, long long nmat, const float2* hls, double2* r_win,
                                   hipStream_t st) {
    const lmmse_plan_desc& d = p.d;
    if (nmat == 0) return hipSuccess;
    ZGemmArgs ga{};
    ga.K = d.K;
    ga.nb = p.nb;
    const long long ms = (long long)d.K * d.N;
    const long long per = (long long)d.Wn * d.Wn;
    ga.A = ZView{hls, 1, ms, (long long)d.M * d.K * d.N, d.N, 1, p.d_starts, 0};
    ga.B = ZView{hls, ms, 1, (long long)d.M * d.K * d.N, d.N, 1, p.d_starts, 1};
    ga.C = ZView{r_win, d.Wn, 1, per * p.nb * d.K, per * p.nb, per, nullptr, 0};
    ga.m = d.Wn;
    ga.n = d.Wn;
    ga.kd = d.M;
    ga.alpha = 1.0 / d.M;
    ga.beta = 0;
    ga.herm = 1;
    return zgemm<float2, float2, double2>(ga, nmat, st);
}

}  // namespace lmmse
