// Sample-covariance estimate for windows wider than the workspace-resident
// design holds (Wn > 256, e.g. the full-band LMMSE of eq. 13 with B = Wn =
// N): the push-through form of the same filter.
//
// With X the Wn x M LS values of a window (column m = antenna m) and
// R = X X^H / M, the block filter W = R_OI (R + lam I)^-1 applied to the
// window's columns gives, by (X X^H / M + lam I)^-1 X = X (X^H X / M + lam I)^-1,
//     W X = [R (R + lam I)^-1 X][O rows] = X_O T,   T = G (G + lam I)^-1 = I - lam (G + lam I)^-1,
// with G = X^H X / M the M x M Gram matrix of the window.  The estimate is
// the same matrix (an exact identity), but the system solved is M x M instead
// of Wn x Wn: for the full band of the paper-sized system 128 x 128 instead
// of 1200 x 1200.  Per (slot, user, block):
//   1. G = X^H X / M: a batched FP64 Hermitian product of the FP32 LS values
//      (exact products, FP64 sums over the Wn window subcarriers);
//   2. -(G + lam I)^-1 by the panel sweep of sample_large.hip;
//   3. T = I + lam (-(G + lam I)^-1);
//   4. h_hat[O_b] = X_O T on the FP32 matrix cores.
#include <algorithm>

#include "zgemm.h"

namespace lmmse {

// T = I + lam S in place, S = -(G + lam I)^-1 as the sweep leaves it.
__global__ __launch_bounds__(256) void pushthrough_t_kernel(double2* a, int n, double lam) {
    double2* am = a + (long long)blockIdx.x * n * n;
    for (int e = threadIdx.x; e < n * n; e += 256) {
        const double2 s = am[e];
        const int i = e / n, j = e - i * n;
        am[e] = make_double2((i == j ? 1.0 : 0.0) + lam * s.x, lam * s.y);
    }
}

size_t pushthrough_bytes(const lmmse_plan_desc& d, long long nmat) {
    return (size_t)nmat * d.M * d.M * sizeof(double2) + sweep_scratch_bytes(d.M, nmat);
}

hipError_t launch_sample_pushthrough(const Plan& p, long long nmat, long long mat0, const float2* hls,
                                     double lam, double2* amat, double2* scratch, float2* out,
                                     hipStream_t st) {
    const lmmse_plan_desc& d = p.d;
    if (nmat == 0) return hipSuccess;
    if (d.M > kMaxPushthroughAntennas) return hipErrorInvalidValue;
    hipError_t e;
    const long long ms = (long long)d.K * d.N, slot = (long long)d.M * d.K * d.N;
    const long long per = (long long)d.M * d.M;
    // G = X^H X / M: A(m, j) = conj(x[m][start + j]), B(j, m') = x[m'][start + j]
    ZGemmArgs ga{};
    ga.K = d.K;
    ga.nb = p.nb;
    ga.A = ZView{hls, ms, 1, slot, d.N, 1, p.d_starts, 1};
    ga.B = ZView{hls, 1, ms, slot, d.N, 1, p.d_starts, 0};
    ga.C = ZView{amat, d.M, 1, per * p.nb * d.K, per * p.nb, per, nullptr, 0};
    ga.m = d.M;
    ga.n = d.M;
    ga.kd = d.Wn;
    ga.alpha = 1.0 / d.M;
    ga.herm = 1;
    if ((e = zgemm<float2, float2, double2>(ga, nmat, st)) != hipSuccess) return e;
    if ((e = launch_sweep_inverse(nmat, mat0, d.M, d.K, p.nb, lam, amat, scratch, p.status, st)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL(pushthrough_t_kernel, dim3((unsigned)nmat), dim3(256), 0, st, amat, d.M, lam);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // out[m][bB + o] = sum_m' T[m'][m] x[m'][bB + o]: A(m, m') = T[m'][m]
    ZGemmArgs gb{};
    gb.K = d.K;
    gb.nb = p.nb;
    gb.A = ZView{amat, 1, d.M, per * p.nb * d.K, per * p.nb, per, nullptr, 0};
    gb.B = ZView{hls, ms, 1, slot, d.N, 1, p.d_bstarts, 0};
    gb.C = ZView{out, ms, 1, slot, d.N, 1, p.d_bstarts, 0};
    gb.m = d.M;
    gb.n = d.B;
    gb.kd = d.M;
    gb.alpha = 1.0;
    return zgemm<double2, float2, float2, float>(gb, nmat, st);
}

}  // namespace lmmse
