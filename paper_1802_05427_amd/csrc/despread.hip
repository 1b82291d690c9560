// LS despreading of code-division pilots (Sec. IV-A-1, eq. 8-9; the paper's
// LS step multiplies by the conjugated unit-modulus pilot instead of
// dividing).  One thread per (slot, antenna, subcarrier): it reads the K pilot
// symbols y[s,m,0..K-1,n] (coalesced along n), undoes the cover code with a
// K-point DFT in registers and writes K LS values
//     h_ls[s,m,k,n] = conj(x_k[n]) / K * sum_t exp(+j 2 pi k t / K) y[s,m,t,n].
#include "dft.h"
#include "internal.h"

namespace lmmse {

template <int K>
__global__ __launch_bounds__(256) void despread_kernel(const float2* __restrict__ y,
                                                       const float2* __restrict__ pilots,
                                                       const float2* __restrict__ twiddle,
                                                       float2* __restrict__ h, int N,
                                                       long long n_ant, float invK) {
    __shared__ float2 tw[K];
    if (threadIdx.x < K) tw[threadIdx.x] = twiddle[threadIdx.x];
    __syncthreads();
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long a = gid / N;
    int n = (int)(gid - a * N);
    if (a >= n_ant) return;
    const float2* yp = y + a * (long long)K * N + n;
    // the pilots are loaded with the symbols, so that all 2K loads are in
    // flight together
    float2 v[K], z[K], x[K];
#pragma unroll
    for (int t = 0; t < K; ++t) v[t] = yp[(long long)t * N];
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = pilots[(long long)k * N + n];
    Dft<K>::run(v, z, tw);
    float2* hp = h + a * (long long)K * N + n;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float2 r = cmulc(z[k], x[k]);
        hp[(long long)k * N] = make_float2(r.x * invK, r.y * invK);
    }
}

// Any K <= 64: direct sum, twiddles in LDS, one output user at a time.
__global__ __launch_bounds__(256) void despread_generic_kernel(const float2* __restrict__ y,
                                                               const float2* __restrict__ pilots,
                                                               const float2* __restrict__ twiddle,
                                                               float2* __restrict__ h, int N, int K,
                                                               long long n_ant, float invK) {
    __shared__ float2 tw[64];
    if (threadIdx.x < K) tw[threadIdx.x] = twiddle[threadIdx.x];
    __syncthreads();
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long a = gid / N;
    int n = (int)(gid - a * N);
    if (a >= n_ant) return;
    const float2* yp = y + a * (long long)K * N + n;
    float2* hp = h + a * (long long)K * N + n;
    for (int k = 0; k < K; ++k) {
        float2 acc = make_float2(0.f, 0.f);
        for (int t = 0; t < K; ++t) {
            float2 v = yp[(long long)t * N];
            float2 w = tw[(k * t) % K];
            acc.x += v.x * w.x - v.y * w.y;
            acc.y += v.x * w.y + v.y * w.x;
        }
        float2 r = cmulc(acc, pilots[(long long)k * N + n]);
        hp[(long long)k * N] = make_float2(r.x * invK, r.y * invK);
    }
}

hipError_t launch_despread(const Plan& p, int slots, const float2* y, const float2* pilots,
                           float2* hls, hipStream_t st) {
    const int K = p.d.K, N = p.d.N;
    const long long n_ant = (long long)slots * p.d.M;
    const long long total = n_ant * N;
    if (total == 0) return hipSuccess;
    const int threads = 256;
    const unsigned grid = (unsigned)((total + threads - 1) / threads);
    const float invK = 1.0f / (float)K;
    switch (K) {
#define LMMSE_DS(KK)                                                                          \
    case KK:                                                                                  \
        hipLaunchKernelGGL(despread_kernel<KK>, dim3(grid), dim3(threads), 0, st, y, pilots,  \
                           p.twiddle, hls, N, n_ant, invK);                                   \
        break;
        LMMSE_DS(1)
        LMMSE_DS(2)
        LMMSE_DS(3)
        LMMSE_DS(4)
        LMMSE_DS(6)
        LMMSE_DS(8)
        LMMSE_DS(12)
        LMMSE_DS(24)
#undef LMMSE_DS
        default:
            hipLaunchKernelGGL(despread_generic_kernel, dim3(grid), dim3(threads), 0, st, y,
                               pilots, p.twiddle, hls, N, K, n_ant, invK);
    }
    return hipGetLastError();
}

}  // namespace lmmse
