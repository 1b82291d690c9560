// Sample-covariance design for windows wider than the register-resident sweep
// of sample.hip holds (160 < Wn <= 256), and the batched inverse it uses
// (also for the caller-correlation design and the push-through form).  The window matrix lives in the
// workspace as FP64 [mat][Wn][Wn] (both triangles):
//
//   1. R = X X^H / M with X = h_ls[s, :, k, I_b]^T: a batched GEMM on the
//      FP32 matrix cores (FP32 products and sums over the M antennas), on the
//      lower tiles only (the upper ones are their mirror), stored as FP64;
//   2. A = R + lam I;
//   3. the Hermitian sweep of all Wn pivots, in panels of 64 pivots K (rest
//      R): sweeping a panel at once maps
//          A_KK -> -A_KK^-1,  A_RK -> A_RK A_KK^-1,  A_KR -> A_KK^-1 A_KR,
//          A_RR -> A_RR - A_RK A_KK^-1 A_KR,
//      which equals sweeping its pivots one by one.  The panel kernel sweeps
//      the 64 x 64 diagonal block and copies the old panel columns P;
//      F = A_RK A_KK^-1 = P A_KK^-1 and the update of A_RR, A += (-1) F P^H,
//      are batched GEMMs (rows of K zero in F and P, so the K rows and
//      columns are left alone); the first stores A_RK = F and A_KR = F^H in
//      place.  After all panels A holds -A^-1;
//   4. W = (I - lam A^-1)[off rows] (FP64 and compact FP32 copies) and,
//      when asked for, A^-1 itself.
#include <algorithm>

#include "split.h"
#include "zgemm.h"

namespace lmmse {

constexpr int kPW = kSweepPanel;
static_assert(kPW == zT, "a panel is one GEMM tile row");

// A = R + lam I on the diagonal of every window.
__global__ __launch_bounds__(256) void add_diag_kernel(double2* a, int Wn, double lam) {
    double2* am = a + (long long)blockIdx.x * Wn * Wn;
    for (int i = threadIdx.x; i < Wn; i += 256) am[(long long)i * Wn + i].x += lam;
}

// Panel step over pivots [k0, k0 + kw) of every window, first part: sweeps
// A_KK into dsw = -A_KK^-1 ([mat][kPW][kPW], zero past kw), writes it to
// A_KK, and copies the old panel columns into P ([mat][Wn][kPW], zero rows
// in K and zero columns >= kw).  F = P A_KK^-1 = P (-dsw) is then a batched
// GEMM that stores A_RK = F and A_KR = F^H.
//
// Thread (w, j) = (tid / 64, tid % 64) of a workgroup of kSwW waves holds
// entries (w + kSwW u, j), u < kSwE, of the 64 x 64 block in registers.
// Sweeping pivot p needs row p and column p as they were before it: their
// holders publish them to LDS (two buffers by the parity of p, so one barrier
// per pivot suffices: a buffer is rewritten two pivots later, after every
// thread has passed the barrier that follows its last read).
constexpr int kSwT = 512;            // threads per window
constexpr int kSwW = kSwT / 64;      // waves
constexpr int kSwE = 64 / kSwW;      // block rows (entries) per thread
__global__ __launch_bounds__(kSwT) void sweep_panel_kernel(double2* a, double2* dsw, double2* pold,
                                                           int Wn, int k0, int kw, int* status,
                                                           long long mat0) {
    static_assert(kPW == 64 && kSwW * kSwE == 64, "thread layout");
    __shared__ double2 rowb[2][kPW], colb[2][kPW];
    __shared__ double2 tsym[kPW / 2][kPW + 1];   // half the block, for its Hermitian part
    const long long mat = blockIdx.x;
    double2* am = a + mat * Wn * Wn;
    const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), j = tid & 63;
    // old panel columns (rows in K zero), rows q0 + w + kSwW v: all loads of
    // a step issued before any store (reads outside use element 0)
    double2* pm = pold + mat * Wn * kPW;
    for (int q0 = 0; q0 < Wn; q0 += 64) {
        double2 v4[kSwE];
        bool ok[kSwE];
#pragma unroll
        for (int v = 0; v < kSwE; ++v) {
            const int i = q0 + w + kSwW * v;
            ok[v] = i < Wn && !(i >= k0 && i < k0 + kw) && j < kw;
            v4[v] = am[ok[v] ? (long long)i * Wn + k0 + j : 0];
        }
#pragma unroll
        for (int v = 0; v < kSwE; ++v) {
            const int i = q0 + w + kSwW * v;
            if (i < Wn) pm[(long long)i * kPW + j] = ok[v] ? v4[v] : make_double2(0.0, 0.0);
        }
    }
    double2 r[kSwE];
    bool okd[kSwE];
#pragma unroll
    for (int u = 0; u < kSwE; ++u) {
        const int i = w + kSwW * u;
        okd[u] = i < kw && j < kw;
        r[u] = am[okd[u] ? (long long)(k0 + i) * Wn + k0 + j : 0];
    }
#pragma unroll
    for (int u = 0; u < kSwE; ++u)
        if (!okd[u]) r[u] = make_double2(0.0, 0.0);
    for (int p = 0; p < kw; ++p) {
        const int buf = p & 1, up = p / kSwW;
        if (w == p % kSwW) {   // row p is entry up of wave p % kSwW (selected by value)
            double2 rp = r[0];
#pragma unroll
            for (int u = 1; u < kSwE; ++u)
                if (up == u) rp = r[u];
            rowb[buf][j] = rp;
        }
        if (j == p) {
#pragma unroll
            for (int u = 0; u < kSwE; ++u) colb[buf][w + kSwW * u] = r[u];
        }
        __syncthreads();
        const double d = rowb[buf][p].x;
        if (!(d > 0.0) || !isfinite(d)) {   // the same d for every thread: uniform exit
            if (tid == 0 && atomicCAS(status, 0, LMMSE_ERR_NOT_PD) == 0)
                status[1] = (int)(mat + mat0);
            return;
        }
        const double invd = 1.0 / d;
        const double2 apj = rowb[buf][j];
        const double2 q = make_double2(apj.x * invd, apj.y * invd);   // row p of the result
        const bool jp = j == p;
#pragma unroll
        for (int u = 0; u < kSwE; ++u) {
            const int i = w + kSwW * u;   // wave-uniform
            const double2 aip = colb[buf][i];
            if (i == p) {
                r[u] = jp ? make_double2(-invd, 0.0) : q;
            } else {   // a_ij - a_ip a_pj / d, and a_ip / d in the pivot column
                const double gx = fma(-aip.x, q.x, fma(aip.y, q.y, r[u].x));
                const double gy = fma(-aip.x, q.y, fma(-aip.y, q.x, r[u].y));
                r[u] = jp ? make_double2(aip.x * invd, aip.y * invd) : make_double2(gx, gy);
            }
        }
    }
    // -A_KK^-1 is Hermitian, but the sweep's rounding is not: the panel
    // product stores A_KR = F^H = (P dsw)^H, which is A_KK^-1 A_KR only for a
    // Hermitian dsw, and the skew part of the rounding grows from panel to
    // panel (a CPU model of a 1200-wide window lost 10 digits over 19
    // panels).  The block is therefore replaced by its Hermitian part.
    // In two halves of 32 block rows (a 64 x 64 buffer would leave room for
    // only two workgroups per CU): entry (i, j) needs (j, i), which the half
    // holding row j provides.
    double2 tr_[kSwE];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int u = 0; u < kSwE; ++u)
            if ((w + kSwW * u) / 32 == h) tsym[(w + kSwW * u) % 32][j] = r[u];
        __syncthreads();
        if (j / 32 == h) {
#pragma unroll
            for (int u = 0; u < kSwE; ++u) tr_[u] = tsym[j % 32][w + kSwW * u];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kSwE; ++u)
        r[u] = make_double2(0.5 * (r[u].x + tr_[u].x), 0.5 * (r[u].y - tr_[u].y));
    double2* dm = dsw + mat * kPW * kPW;
#pragma unroll
    for (int u = 0; u < kSwE; ++u) {
        const int i = w + kSwW * u;
        dm[i * kPW + j] = r[u];
        if (i < kw && j < kw) am[(long long)(k0 + i) * Wn + k0 + j] = r[u];
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

// A -> -A^-1 of nmat Hermitian n x n matrices [mat][n][n] (both triangles)
// after adding lam to their diagonals: the panel sweep described at the top
// of this file.  The batch index decomposes as (slot * K + user) * nb +
// block, as in every batched product here (only the strides depend on it).
// scratch: sweep_scratch_bytes(n, nmat).  A non-positive pivot records
// LMMSE_ERR_NOT_PD with matrix mat0 + mat in status.
hipError_t launch_sweep_inverse(long long nmat, long long mat0, int n, int K, int nb, double lam,
                                double2* amat, double2* scratch, int* status, hipStream_t st) {
    if (nmat == 0) return hipSuccess;
    hipError_t e;
    hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)nmat), dim3(256), 0, st, amat, n, lam);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ZGemmArgs ga{};
    ga.K = K;
    ga.nb = nb;
    const long long per = (long long)n * n;
    // scratch: P [nmat][n][kPW], then -A_KK^-1 [nmat][kPW][kPW]
    double2* pold = scratch;
    double2* dsw = pold + nmat * n * kPW;
    const long long pp = (long long)n * kPW, dd = (long long)kPW * kPW;
    for (int k0 = 0; k0 < n; k0 += kPW) {
        const int kw = std::min(kPW, n - k0);
        hipLaunchKernelGGL(sweep_panel_kernel, dim3((unsigned)nmat), dim3(kSwT), 0, st, amat, dsw,
                           pold, n, k0, kw, status, mat0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // F = P A_KK^-1 = -P dsw, stored in place as A_RK = F (the panel's
        // columns) and A_KR = F^H (its rows).  Rows of K vanish with P's: the
        // panel's tile row is left out, which keeps A_KK as the sweep wrote it.
        ga.skip_tile = k0 / kPW;
        ga.A = ZView{pold, kPW, 1, pp * nb * K, pp * nb, pp, nullptr, 0};
        ga.B = ZView{dsw, kPW, 1, dd * nb * K, dd * nb, dd, nullptr, 0};
        ga.C = ZView{amat + k0, n, 1, per * nb * K, per * nb, per, nullptr, 0};
        ga.T = ZView{amat + (long long)k0 * n, n, 1, per * nb * K, per * nb, per, nullptr, 0};
        ga.tcopy = 1;
        ga.m = n;
        ga.n = kw;
        ga.kd = kw;
        ga.alpha = -1.0;
        ga.beta = 0;
        ga.herm = 0;
        if ((e = zgemm<double2, double2, double2>(ga, nmat, st)) != hipSuccess) return e;
        ga.tcopy = 0;
        // A += (-1) F P^H over the matrix but the panel's tile row and column,
        // where F P^H vanishes (F and P are zero on the panel's rows); F is
        // read from the panel's columns, which this product does not write
        ga.A = ZView{amat + k0, n, 1, per * nb * K, per * nb, per, nullptr, 0};
        ga.B = ZView{pold, 1, kPW, pp * nb * K, pp * nb, pp, nullptr, 1};
        ga.C = ZView{amat, n, 1, per * nb * K, per * nb, per, nullptr, 0};
        ga.m = n;
        ga.n = n;
        ga.kd = kw;
        ga.alpha = -1.0;
        ga.beta = 1;
        ga.herm = 1;   // F P^H = A_RK A_KK^-1 A_RK^H is Hermitian
        if ((e = zgemm<double2, double2, double2>(ga, nmat, st)) != hipSuccess) return e;
        ga.skip_tile = -1;
    }
    return hipSuccess;
}

hipError_t launch_large_filters(long long nmat, double2* amat, const int* offsets, int B, int Wn,
                                int nb, double lam, double2* w64, bool negate, hipStream_t st) {
    if (nmat == 0) return hipSuccess;
    hipLaunchKernelGGL(large_filters_kernel, dim3((unsigned)nmat), dim3(256), 0, st, amat, offsets, B,
                       Wn, nb, lam, w64, nullptr, nullptr, nullptr, 0, negate ? 1 : 0);
    return hipGetLastError();
}

size_t sweep_scratch_bytes(int Wn, long long nmat) {
    return (size_t)nmat * ((size_t)Wn * kPW + (size_t)kPW * kPW) * sizeof(double2);
}

size_t large_design_bytes(const lmmse_plan_desc& d, long long nmat) {
    return (size_t)nmat * d.Wn * d.Wn * sizeof(double2) + sweep_scratch_bytes(d.Wn, nmat);
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
    // FP32 matrix-core products and sums, stored as FP64 for the sweep
    if ((e = zgemm<float2, float2, double2, float>(ga, nmat, st)) != hipSuccess) return e;
    ga.herm = 0;
    if ((e = launch_sweep_inverse(nmat, mat0, Wn, d.K, p.nb, lam, amat, scratch, p.status, st)) !=
        hipSuccess)
        return e;
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
