// FP64 filter design on the GPU (eq. 13 / eq. 17 per block, Sec. IV-B).
//
// Fixed design: the window correlation R_II is the same Hermitian Toeplitz
// matrix for every block (the correlation depends only on the subcarrier
// difference, eq. 16), so one Cholesky factorisation A = R_II + lam I = L L^H
// serves all blocks.  Solving A X = R_II gives X = A^-1 R_II, and the filter
// of a block whose outputs sit at rows off..off+B-1 of its window is
//     W = R_OI A^-1 = (A^-1 R_IO)^H,   W[i][j] = conj(X[j][off + i]).
// Matrices are column-major (element (i, j) at i + j*n).
#include "internal.h"

namespace lmmse {

__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 zmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }

// r_d and d r_d / d tau for d = 0..n-1.
//  uniform (eq. 16):  r_d = (1 - e^{-j a}) / (j a),  a = 2 pi L d / N_fft
//                         = sin(a)/a - j (2 sin^2(a/2))/a
//  exponential:       r_d = sum_l p_l e^{-j 2 pi l d / N_fft},  p_l = e^{-l/tau} / S
//                     dr_d/dtau = sum_l p_l (l - lbar) / tau^2 e^{-j 2 pi l d / N_fft}
__global__ void rd_kernel(double2* rd, int n, int rsource, double L, double tau, int taps,
                          int N_fft) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    double2 r = make_double2(0.0, 0.0), dr = make_double2(0.0, 0.0);
    if (rsource == LMMSE_R_UNIFORM) {
        if (d == 0) {
            r = make_double2(1.0, 0.0);
        } else {
            const double a = 2.0 * M_PI * L * (double)d / (double)N_fft;
            const double sh = sin(0.5 * a);
            r = make_double2(sin(a) / a, -2.0 * sh * sh / a);
        }
    } else {
        double S = 0.0, S1 = 0.0;
        for (int l = 0; l < taps; ++l) {
            const double w = exp(-(double)l / tau);
            S += w;
            S1 += (double)l * w;
        }
        const double lbar = S1 / S;
        for (int l = 0; l < taps; ++l) {
            const double p = exp(-(double)l / tau) / S;
            const long long m = ((long long)l * d) % N_fft;
            double sn, cs;
            sincospi(2.0 * (double)m / (double)N_fft, &sn, &cs);
            r.x += p * cs;
            r.y -= p * sn;
            const double dp = p * ((double)l - lbar) / (tau * tau);
            dr.x += dp * cs;
            dr.y -= dp * sn;
        }
    }
    rd[d] = r;
    rd[n + d] = dr;
}

// A = R_II + lam I and F = R_II (column-major, n x n) from r_d.
__global__ void toeplitz_kernel(const double2* __restrict__ rd, double2* __restrict__ A,
                                double2* __restrict__ F, int n, double lam) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * n) return;
    const int i = (int)(idx % n), j = (int)(idx / n);
    const int dd = i - j;
    const double2 r = dd >= 0 ? rd[dd] : zconj(rd[-dd]);
    F[idx] = r;
    A[idx] = i == j ? make_double2(r.x + lam, 0.0) : r;
}

// In-place lower Cholesky of one n x n Hermitian matrix per workgroup
// (column-major, right-looking; the pivot column is cached in LDS).
// On a non-positive or non-finite pivot the status word gets
// LMMSE_ERR_NOT_PD and info = info_base + blockIdx.x (first failure wins).
__global__ __launch_bounds__(1024) void chol_kernel(double2* A, long long strideA, int n,
                                                    int* status, int info_base) {
    extern __shared__ double2 col[];   // n entries
    __shared__ double piv_s;
    __shared__ int bad;
    A += (long long)blockIdx.x * strideA;
    const int tid = threadIdx.x, ti = tid & 31, tp = tid >> 5;
    if (tid == 0) bad = 0;
    for (int j = 0; j < n; ++j) {
        __syncthreads();
        if (tid == 0) {
            const double dj = A[j + (long long)j * n].x;
            if (!(dj > 0.0) || !isfinite(dj)) {
                bad = 1;
                if (atomicCAS(status, 0, LMMSE_ERR_NOT_PD) == 0) status[1] = info_base + blockIdx.x;
            }
            piv_s = sqrt(dj);
            A[j + (long long)j * n] = make_double2(piv_s, 0.0);
        }
        __syncthreads();
        if (bad) return;
        const double inv = 1.0 / piv_s;
        for (int i = j + 1 + tid; i < n; i += blockDim.x) {
            double2 v = A[i + (long long)j * n];
            v = make_double2(v.x * inv, v.y * inv);
            A[i + (long long)j * n] = v;
            col[i] = v;
        }
        __syncthreads();
        for (int p = j + 1 + tp; p < n; p += 32) {
            const double2 cp = col[p];
            double2* Ap = A + (long long)p * n;
            for (int i = p + ti; i < n; i += 32) {
                const double2 u = zmulc(col[i], cp);
                Ap[i] = zsub(Ap[i], u);
            }
        }
    }
}

// Solve A X = Y in place for the columns of Y (column-major n x nrhs),
// given the lower Cholesky factor of A.  Each workgroup handles NC columns
// staged in LDS; 256 threads = NC columns x (256/NC) row lanes.
__global__ __launch_bounds__(256) void chol_solve_kernel(const double2* __restrict__ Lf, double2* Y,
                                                         int n, int nrhs, int NC) {
    extern __shared__ double2 ys[];   // [NC][n]
    const int tid = threadIdx.x;
    const int R = 256 / NC;
    const int c = tid / R, rl = tid % R;
    const int col = blockIdx.x * NC + c;
    const bool live = col < nrhs;
    double2* yl = ys + (long long)c * n;
    if (live)
        for (int i = rl; i < n; i += R) yl[i] = Y[i + (long long)col * n];
    // forward: L z = y.  Row i is divided by L[i][i] right after its last
    // update (at step i-1), so step j only reads the finished z_j.
    __syncthreads();
    if (live && rl == 0) {
        const double d = Lf[0].x;
        yl[0] = make_double2(yl[0].x / d, yl[0].y / d);
    }
    for (int j = 0; j < n; ++j) {
        __syncthreads();
        if (live) {
            const double2 yj = yl[j];
            const double2* Lj = Lf + (long long)j * n;
            for (int i = j + 1 + rl; i < n; i += R) {
                double2 v = zsub(yl[i], zmul(Lj[i], yj));
                if (i == j + 1) {
                    const double d = Lf[i + (long long)i * n].x;
                    v = make_double2(v.x / d, v.y / d);
                }
                yl[i] = v;
            }
        }
    }
    // backward: L^H x = z, same scheme from the bottom row up.
    __syncthreads();
    if (live && rl == 0) {
        const double d = Lf[(n - 1) + (long long)(n - 1) * n].x;
        yl[n - 1] = make_double2(yl[n - 1].x / d, yl[n - 1].y / d);
    }
    for (int j = n - 1; j >= 0; --j) {
        __syncthreads();
        if (live) {
            const double2 xj = yl[j];
            for (int i = rl; i < j; i += R) {
                double2 v = zsub(yl[i], zmul(zconj(Lf[j + (long long)i * n]), xj));
                if (i == j - 1) {
                    const double d = Lf[i + (long long)i * n].x;
                    v = make_double2(v.x / d, v.y / d);
                }
                yl[i] = v;
            }
        }
    }
    __syncthreads();
    if (live)
        for (int i = rl; i < n; i += R) Y[i + (long long)col * n] = yl[i];
}

// W_c[i][j] = conj(X[j][off_c + i])  (X = A^-1 R_II, column-major n x n).
__global__ void extract_kernel(const double2* __restrict__ X, const int* __restrict__ class_off,
                               double2* __restrict__ w, int n_classes, int B, int n) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)B * n;
    if (idx >= per * n_classes) return;
    const int c = (int)(idx / per);
    const long long r = idx % per;
    const int i = (int)(r / n), j = (int)(r % n);
    w[idx] = zconj(X[j + (long long)(class_off[c] + i) * n]);
}

// Real embedding element Wr[r][kr] of filter w (B x Wn complex).
__device__ __forceinline__ double wreal(const double2* w, int B, int Wn, int r, int kr) {
    const int a = r >> 1, ra = r & 1, jj = kr >> 1, rj = kr & 1;
    if (a >= B || jj >= Wn) return 0.0;
    const double2 v = w[(long long)a * Wn + jj];
    if (ra == 0) return rj == 0 ? v.x : -v.y;
    return rj == 0 ? v.y : v.x;
}

__global__ void pack_f32_kernel(const double2* __restrict__ w64, float4* __restrict__ bank,
                                int n_classes, int B, int Wn, int G8, int Rpad) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)n_classes * G8 * Rpad * 4;
    if (idx >= total) return;
    const int q = (int)(idx & 3);
    long long t = idx >> 2;
    const int r = (int)(t % Rpad);
    t /= Rpad;
    const int g = (int)(t % G8);
    const int c = (int)(t / G8);
    const double2* w = w64 + (long long)c * B * Wn;
    const int k0 = 16 * g + 4 * q;
    bank[idx] = make_float4((float)wreal(w, B, Wn, r, k0), (float)wreal(w, B, Wn, r, k0 + 1),
                            (float)wreal(w, B, Wn, r, k0 + 2), (float)wreal(w, B, Wn, r, k0 + 3));
}

// Round-to-nearest-even conversions (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// hi = round(x), lo = round((x - hi) * lo_scale) in BF16 (is_fp16 = 0) or FP16.
__global__ void pack_split_kernel(const double2* __restrict__ w64, uint16_t* __restrict__ hi,
                                  uint16_t* __restrict__ lo, int n_classes, int B, int Wn, int G16,
                                  int Rpad, int is_fp16, double lo_scale) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)n_classes * G16 * Rpad * 32;
    if (idx >= total) return;
    const int e = (int)(idx & 7);
    const int kq = (int)((idx >> 3) & 3);
    long long t = idx >> 5;
    const int r = (int)(t % Rpad);
    t /= Rpad;
    const int g = (int)(t % G16);
    const int c = (int)(t / G16);
    const double x = wreal(w64 + (long long)c * B * Wn, B, Wn, r, 32 * g + 8 * kq + e);
    if (is_fp16) {
        const _Float16 h = (_Float16)x;
        const _Float16 l = (_Float16)((x - (double)h) * lo_scale);
        hi[idx] = __builtin_bit_cast(uint16_t, h);
        lo[idx] = __builtin_bit_cast(uint16_t, l);
    } else {
        const uint16_t h = f32_to_bf16((float)x);
        const uint16_t l = f32_to_bf16((float)((x - (double)bf16_to_f32(h)) * lo_scale));
        hi[idx] = h;
        lo[idx] = l;
    }
}

static int solve_cols_per_wg(int n) {
    int nc = 16;
    while (nc > 1 && (long long)nc * n * 16 > 65536) nc >>= 1;
    return nc;
}

hipError_t launch_chol(double2* A, long long strideA, int n, int nmat, int* status, int info_base,
                       hipStream_t st) {
    hipLaunchKernelGGL(chol_kernel, dim3(nmat), dim3(1024), (size_t)n * sizeof(double2), st, A,
                       strideA, n, status, info_base);
    return hipGetLastError();
}

hipError_t launch_chol_solve(const double2* L, double2* Y, int n, int nrhs, hipStream_t st) {
    const int nc = solve_cols_per_wg(n);
    const unsigned grid = (unsigned)((nrhs + nc - 1) / nc);
    hipLaunchKernelGGL(chol_solve_kernel, dim3(grid), dim3(256), (size_t)nc * n * sizeof(double2),
                       st, L, Y, n, nrhs, nc);
    return hipGetLastError();
}

hipError_t launch_pack_banks(Plan& p, hipStream_t st) {
    const int B = p.d.B, Wn = p.d.Wn;
    {
        const long long total = (long long)p.n_classes * p.G8 * p.Rpad * 4;
        hipLaunchKernelGGL(pack_f32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                           p.w64, p.wf32, p.n_classes, B, Wn, p.G8, p.Rpad);
    }
    if (p.whi) {
        const long long total = (long long)p.n_classes * p.G16 * p.Rpad * 32;
        hipLaunchKernelGGL(pack_split_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                           st, p.w64, p.whi, p.wlo, p.n_classes, B, Wn, p.G16, p.Rpad,
                           p.d.precision == LMMSE_FP16X3 ? 1 : 0, (double)p.lo_scale);
    }
    return hipGetLastError();
}

hipError_t launch_fixed_design(Plan& p, double tau, double sigma2, hipStream_t st) {
    const int n = p.d.Wn;
    const double lam = sigma2 / p.d.K;
    hipLaunchKernelGGL(rd_kernel, dim3((n + 127) / 128), dim3(128), 0, st, p.rd, n, p.d.rsource,
                       p.d.L, tau, p.d.taps, p.d.N_fft);
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(toeplitz_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, p.rd,
                       p.chol, p.fmat, n, lam);
    hipError_t e = launch_chol(p.chol, 0, n, 1, p.status, 0, st);
    if (e != hipSuccess) return e;
    e = launch_chol_solve(p.chol, p.fmat, n, n, st);
    if (e != hipSuccess) return e;
    const long long tot = (long long)p.n_classes * p.d.B * n;
    hipLaunchKernelGGL(extract_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       p.fmat, p.d_class_off, p.w64, p.n_classes, p.d.B, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_pack_banks(p, st);
}

}  // namespace lmmse
