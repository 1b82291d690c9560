// Sample-covariance design for windows wider than the register-resident sweep
// of sample.hip holds (160 < Wn <= 256), and the batched inverse it uses
// (also for the caller-correlation design and the push-through form).  The window matrix lives in the
// workspace as FP64 [mat][Wn][Wn] (both triangles):
//
//   1. R = X X^H / M with X = h_ls[s, :, k, I_b]^T: a batched GEMM on the
//      FP32 matrix cores (FP32 products and sums over the M antennas), on the
//      lower tiles only (the upper ones are their mirror), stored as FP64;
//   2. A = R + lam I;
//   3. the Hermitian sweep of all Wn pivots: for Wn <= 208 in one launch
//      with the matrix held on one compute unit, which also forms steps 1,
//      2 and 4 itself (resident_inverse.hip); wider, in panels of 64 pivots
//      K (rest R): sweeping a panel at once maps
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
// holders publish them to LDS (two buffers by the parity of the step, so one
// barrier per step suffices: a buffer is rewritten two steps later, after
// every thread has passed the barrier that follows its last read).  Pivots
// are swept in pairs (below).
constexpr int kSwT = 512;            // threads per window
constexpr int kSwW = kSwT / 64;      // waves
constexpr int kSwE = 64 / kSwW;      // block rows (entries) per thread
__global__ __launch_bounds__(kSwT) void sweep_panel_kernel(double2* a, double2* dsw, double2* pold,
                                                           int Wn, int k0, int kw, int* status,
                                                           long long mat0) {
    static_assert(kPW == 64 && kSwW * kSwE == 64, "thread layout");
    // One LDS area: the pivot rows and columns during the sweep ([step
    // parity][pivot of the pair][64]), then half the block for its Hermitian
    // part (37 KB in all, so four workgroups fit a CU).
    __shared__ double2 lds[kPW / 2 * (kPW + 1)];
    static_assert(4 * 2 * kPW <= kPW / 2 * (kPW + 1), "pivot buffers fit the area");
    double2(*rowb)[2][kPW] = reinterpret_cast<double2(*)[2][kPW]>(lds);
    double2(*colb)[2][kPW] = reinterpret_cast<double2(*)[2][kPW]>(lds + 2 * 2 * kPW);
    double2(*tsym)[kPW + 1] = reinterpret_cast<double2(*)[kPW + 1]>(lds);
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
    // Pivots two at a time, with one barrier for the pair: the step applies
    // the sweep of p and then that of p+1 in closed form, in the same order of
    // operations (p's quotients, then p+1's pivot as the Schur complement
    // d2 = c - |b|^2 / a), which keeps the rounding of single pivots; forming
    // the 2 x 2 inverse of [[a, b], [conj b, c]] instead loses accuracy as
    // the windows' conditioning grows (about 20 dB at 30 dB SNR in a CPU
    // model).  An odd last pivot is swept alone.  The step's pivot rows and
    // columns are published to LDS (two buffers by the parity of the step,
    // so one barrier per step suffices).
    int step = 0, p = 0;
    for (; p + 1 < kw; p += 2, ++step) {
        const int buf = step & 1, up = p / kSwW;   // rows p, p+1: entry up of waves p%8, p%8+1
        if (w == p % kSwW || w == (p + 1) % kSwW) {
            double2 rp = r[0];
#pragma unroll
            for (int u = 1; u < kSwE; ++u)
                if (up == u) rp = r[u];
            rowb[buf][w == p % kSwW ? 0 : 1][j] = rp;
        }
        if (j == p || j == p + 1) {
#pragma unroll
            for (int u = 0; u < kSwE; ++u) colb[buf][j - p][w + kSwW * u] = r[u];
        }
        __syncthreads();
        const double a = rowb[buf][0][p].x, c = rowb[buf][1][p + 1].x;
        const double2 b = rowb[buf][0][p + 1];   // a_{p,p+1}
        const double inva = 1.0 / a;
        const double2 ba = make_double2(b.x * inva, b.y * inva);   // row p+1 after pivot p, col p+1
        const double d2 = c - (b.x * ba.x + b.y * ba.y);
        if (!(a > 0.0) || !isfinite(a) || !(d2 > 0.0) || !isfinite(d2)) {   // uniform
            if (tid == 0 && atomicCAS(status, 0, LMMSE_ERR_NOT_PD) == 0)
                status[1] = (int)(mat + mat0);
            return;
        }
        const double invd2 = 1.0 / d2;
        const double2 cb = make_double2(ba.x * invd2, -ba.y * invd2);   // conj(b) / (a d2)
        // column j outside the pair: q = a_pj / a, t1 = (a_{p+1,j} - conj(b) q) / d2,
        // t0 = q - (b / a) t1 (rows p+1 and p of the result)
        const double2 apj = rowb[buf][0][j], bpj = rowb[buf][1][j];
        const double2 q = make_double2(apj.x * inva, apj.y * inva);
        const double2 bq = make_double2(bpj.x - (b.x * q.x + b.y * q.y), bpj.y - (b.x * q.y - b.y * q.x));
        const double2 t1 = make_double2(bq.x * invd2, bq.y * invd2);
        const double2 t0 = make_double2(q.x - (ba.x * t1.x - ba.y * t1.y), q.y - (ba.x * t1.y + ba.y * t1.x));
        const bool j0 = j == p, j1 = j == p + 1;
        // Rows outside the pair take one formula in every column, rs a_ij -
        // x0 ql - x1 tl, with per-lane coefficients set once per step: off the
        // pair's columns rs = 1, ql = q, tl = t1 (a_ij - x0 q - x1 t1); in
        // column p, A_iK A_KK^-1's first column x0 / a - x1 conj(b) / (a d2)
        // (rs = 0, ql = -1/a, tl = conj(b) / (a d2)); in column p+1, x1 / d2
        // (rs = 0, ql = 0, tl = -1/d2).  Branching per lane instead would run
        // all three forms in every wave.
        const double rs = (j0 || j1) ? 0.0 : 1.0;
        const double2 ql = j0 ? make_double2(-inva, 0.0) : j1 ? make_double2(0.0, 0.0) : q;
        const double2 tl = j0 ? cb : j1 ? make_double2(-invd2, 0.0) : t1;
#pragma unroll
        for (int u = 0; u < kSwE; ++u) {
            const int i = w + kSwW * u;   // wave-uniform
            if (i == p) {
                r[u] = j0 ? make_double2(-inva - (ba.x * ba.x + ba.y * ba.y) * invd2, 0.0)
                     : j1 ? make_double2(ba.x * invd2, ba.y * invd2) : t0;
            } else if (i == p + 1) {
                r[u] = j0 ? cb : j1 ? make_double2(-invd2, 0.0) : t1;
            } else {
                // x0 = a_ip; x1 = a_{i,p+1} - a_ip b / a after pivot p
                const double2 x0 = colb[buf][0][i], x1o = colb[buf][1][i];
                const double2 x1 = make_double2(x1o.x - (x0.x * ba.x - x0.y * ba.y),
                                                x1o.y - (x0.x * ba.y + x0.y * ba.x));
                double gx = fma(-x0.x, ql.x, fma(x0.y, ql.y, rs * r[u].x));
                double gy = fma(-x0.x, ql.y, fma(-x0.y, ql.x, rs * r[u].y));
                gx = fma(-x1.x, tl.x, fma(x1.y, tl.y, gx));
                gy = fma(-x1.x, tl.y, fma(-x1.y, tl.x, gy));
                r[u] = make_double2(gx, gy);
            }
        }
    }
    if (p < kw) {   // odd last pivot, alone
        const int buf = step & 1, up = p / kSwW;
        if (w == p % kSwW) {
            double2 rp = r[0];
#pragma unroll
            for (int u = 1; u < kSwE; ++u)
                if (up == u) rp = r[u];
            rowb[buf][0][j] = rp;
        }
        if (j == p) {
#pragma unroll
            for (int u = 0; u < kSwE; ++u) colb[buf][0][w + kSwW * u] = r[u];
        }
        __syncthreads();
        const double d = rowb[buf][0][p].x;
        if (!(d > 0.0) || !isfinite(d)) {
            if (tid == 0 && atomicCAS(status, 0, LMMSE_ERR_NOT_PD) == 0)
                status[1] = (int)(mat + mat0);
            return;
        }
        const double invd = 1.0 / d;
        const double2 apj = rowb[buf][0][j];
        const double2 q = make_double2(apj.x * invd, apj.y * invd);   // row p of the result
        const bool jp = j == p;
#pragma unroll
        for (int u = 0; u < kSwE; ++u) {
            const int i = w + kSwW * u;
            const double2 aip = colb[buf][0][i];
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
    __syncthreads();   // every read of the pivot buffers is done
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
    // FP32 and split filters: B x W16 per window in the chunk-major order of
    // split_w_index, the pad columns Wn..W16-1 zero
    const int w16 = (Wn + 15) & ~15;
    const long long wb = mat * B * (long long)w16;
    for (int e = threadIdx.x; e < B * w16; e += 256) {
        const int o = e / w16, j = e - o * w16;
        if (j >= Wn) {
            if (w32) w32[split_w_index(wb, B, o, j)] = make_float2(0.f, 0.f);
            continue;
        }
        const double2 s = am[(long long)(off + o) * Wn + j];
        const double2 w = make_double2((off + o == j ? 1.0 : 0.0) + lam * s.x, lam * s.y);
        if (w64) w64[(mat * B + o) * Wn + j] = w;
        if (w32) w32[split_w_index(wb, B, o, j)] = make_float2((float)w.x, (float)w.y);
        if (whi) store_split_w(whi, wlo, mat * B * (long long)w16, B, o, j, Wn, w16, w, fp16);
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
    // a matrix that one compute unit holds whole: the register-resident form
    if (resident_inverse_fits(n)) return launch_resident_inverse(nmat, mat0, n, lam, amat, status, st);
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
    if (resident_inverse_fits(Wn)) return 0;   // no panel operands
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
    if (resident_inverse_fits(Wn))   // covariance, sweep and filters in one kernel per window
        return launch_resident_design(p, nmat, mat0, hls, lam, amat, w64, w32, whi, wlo, want_ainv, st);
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
