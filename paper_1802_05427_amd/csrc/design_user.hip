// Block filters from a caller-supplied subcarrier correlation (eq. 13 per
// block of Sec. IV-B with R_HH given, e.g. measured or computed offline as
// the paper's weights are, Sec. IV-C).  R is any N x N Hermitian matrix, so
// the windows are not Toeplitz and every block has its own filter:
//     W_b = R[O_b, I_b] (R[I_b, I_b] + lam I)^-1 = (I - lam A_b^-1)[off_b rows],
// A_b = R[I_b, I_b] + lam I, lam = sigma2 / K, FP64.  The windows are copied
// out of R once (the plan keeps them, so a new sigma2 redesigns without R);
// A_b^-1 is kept (row-major) for the backward pass.  Windows up to 160 use
// the register-resident sweep of sample.hip, wider ones the panel sweep of
// sample_large.hip in the plan's scratch.
#include "internal.h"

namespace lmmse {

// rwin[b][i][j] = r[(start_b + i) * N + start_b + j]
__global__ __launch_bounds__(256) void gather_windows_kernel(const double2* __restrict__ r, int N,
                                                             const int* __restrict__ starts, int Wn,
                                                             double2* __restrict__ rwin) {
    const int b = blockIdx.y;
    const long long per = (long long)Wn * Wn;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= per) return;
    const int i = (int)(e / Wn), j = (int)(e - (long long)i * Wn);
    const long long s = starts[b];
    rwin[b * per + e] = r[(s + i) * N + s + j];
}

size_t user_corr_scratch_bytes(const lmmse_plan_desc& d) {
    return d.Wn > kMaxSampleWindowReg ? sweep_scratch_bytes(d.Wn, d.N / d.B) : 0;
}

hipError_t launch_user_corr_gather(Plan& p, const double2* r, hipStream_t st) {
    const long long per = (long long)p.d.Wn * p.d.Wn;
    hipLaunchKernelGGL(gather_windows_kernel, dim3((unsigned)((per + 255) / 256), (unsigned)p.nb),
                       dim3(256), 0, st, r, p.d.N, p.d_starts, p.d.Wn, p.rwin);
    return hipGetLastError();
}

hipError_t launch_user_corr_design(Plan& p, double sigma2, hipStream_t st) {
    const double lam = sigma2 / p.d.K;
    const int Wn = p.d.Wn;
    hipError_t e;
    if (Wn <= kMaxSampleWindowReg) {
        e = launch_batched_filters(p, p.nb, p.rwin, lam, p.w64, p.ainv, st);
    } else {
        const size_t bytes = (size_t)p.nb * Wn * Wn * sizeof(double2);
        if ((e = hipMemcpyAsync(p.ainv, p.rwin, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return e;
        if ((e = launch_sweep_inverse(p.nb, 0, Wn, 1, p.nb, lam, p.ainv, p.dwork, p.status, st)) !=
            hipSuccess)
            return e;
        e = launch_large_filters(p.nb, p.ainv, p.d_offsets, p.d.B, Wn, p.nb, lam, p.w64, true, st);
    }
    if (e != hipSuccess) return e;
    return launch_pack_banks(p, st);
}

}  // namespace lmmse
