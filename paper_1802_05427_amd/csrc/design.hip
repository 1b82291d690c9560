// FP64 filter design on the GPU (eq. 13 / eq. 17 per block, Sec. IV-B).
//
// Fixed design: the window correlation R_II is the same Hermitian Toeplitz
// matrix for every block (the correlation depends only on the subcarrier
// difference, eq. 16), and so is A = R_II + lam I.  Since R_II A^-1 =
// (A - lam I) A^-1 = I - lam A^-1, the filter of a block whose outputs sit at
// rows off..off+B-1 of its window is
//     W = R_OI A^-1 = (I - lam A^-1)[off : off+B, :].
// A^-1 of the Hermitian positive definite Toeplitz A is formed in O(n^2):
// the Levinson-Durbin recursion gives its first column x, and the displacement
// structure of the inverse of a Toeplitz matrix (Gohberg-Semencul) gives every
// other entry along its diagonal:
//     Ainv[i][j] = Ainv[i-1][j-1] + (x_i conj(x_j) - y_{i-1} conj(y_{j-1})) / x_0,
//     y_k = conj(x_{n-1-k})  (the last column).
// A^-1 is kept for the backward pass.  Matrices are column-major (element
// (i, j) at i + j*n).
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

// r_d and d r_d / d tau for d = 0..n-1, one wave per d.
//  uniform (eq. 16):  r_d = (1 - e^{-j a}) / (j a),  a = 2 pi L d / N_fft
//                         = sin(a)/a - j (2 sin^2(a/2))/a
//  exponential:       r_d = sum_l p_l e^{-j 2 pi l d / N_fft},  p_l = e^{-l/tau} / S
//                     dr_d/dtau = sum_l p_l (l - lbar) / tau^2 e^{-j 2 pi l d / N_fft}
// The tap sums are split over the lanes and reduced in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// 64-lane sum with the result in every lane, in a fixed order: within each
// 16-lane row by DPP moves (the quad swaps 1-0-3-2 and 2-3-0-1, then the
// half-row and row mirrors, each an exchange with lanes that hold the other
// half of the partial sum), then the four row sums read from lanes 0, 16, 32
// and 48.  No LDS round trip, unlike a shuffle.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_move<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);   // row_half_mirror
    v += dpp_move<0x140>(v);   // row_mirror
    return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
}

__global__ __launch_bounds__(64) void rd_kernel(double2* rd, int n, int rsource, double L, double tau,
                                                int taps, int N_fft) {
    const int d = blockIdx.x, lane = threadIdx.x;
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
        for (int l = lane; l < taps; l += 64) {
            const double w = exp(-(double)l / tau);
            S += w;
            S1 += (double)l * w;
        }
        S = wave_sum(S);
        S1 = wave_sum(S1);
        const double lbar = S1 / S;
        double rx = 0.0, ry = 0.0, dx = 0.0, dy = 0.0;
        for (int l = lane; l < taps; l += 64) {
            const double p = exp(-(double)l / tau) / S;
            const long long m = ((long long)l * d) % N_fft;
            double sn, cs;
            sincospi(2.0 * (double)m / (double)N_fft, &sn, &cs);
            rx += p * cs;
            ry -= p * sn;
            const double dp = p * ((double)l - lbar) / (tau * tau);
            dx += dp * cs;
            dy -= dp * sn;
        }
        r = make_double2(wave_sum(rx), wave_sum(ry));
        dr = make_double2(wave_sum(dx), wave_sum(dy));
    }
    if (lane == 0) {
        rd[d] = r;
        rd[n + d] = dr;
    }
}

// Levinson-Durbin on A[i][j] = a_{i-j}, a_d = r_d + lam delta_d (a_{-d} =
// conj(a_d)), giving x = A^-1 e_0.  One wave; LDS holds
// a_d and two copies of the predictor.  Predictor of order k: A_{k+1} [1; p]
// = [P_k; 0], p^(k)_i = p^(k-1)_i + kap conj(p^(k-1)_{k-i}), p^(k)_k = kap,
// kap = -(a_k + sum_{i<k} p_i a_{k-i}) / P_{k-1}, P_k = P_{k-1} (1 - |kap|^2).
// A non-positive P (A not positive definite) sets LMMSE_ERR_NOT_PD.
__global__ __launch_bounds__(64) void toeplitz_inverse_kernel(const double2* __restrict__ rd, int n,
                                                              double lam, double2* __restrict__ xout,
                                                              int* status) {
    extern __shared__ double2 sh[];
    double2* av = sh;            // a_d
    double2* p0 = sh + n;        // predictor buffers
    double2* p1 = sh + 2 * n;
    const int tid = threadIdx.x;
    for (int d = tid; d < n; d += 64) {
        const double2 r = rd[d];
        av[d] = d == 0 ? make_double2(r.x + lam, 0.0) : r;
        p0[d] = make_double2(0.0, 0.0);
        p1[d] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    double P = av[0].x;
    bool ok = P > 0.0 && isfinite(P);
    double2* cur = p0;
    double2* nxt = p1;
    for (int k = 1; k < n && ok; ++k) {
        double sr = 0.0, si = 0.0;
        for (int i = 1 + tid; i < k; i += 64) {
            const double2 u = zmul(cur[i], av[k - i]);
            sr += u.x;
            si += u.y;
        }
        sr = wave_sum_dpp(sr);
        si = wave_sum_dpp(si);
        const double2 delta = make_double2(av[k].x + sr, av[k].y + si);
        const double2 kap = make_double2(-delta.x / P, -delta.y / P);
        for (int i = 1 + tid; i < k; i += 64) nxt[i] = zadd(cur[i], zmul(kap, zconj(cur[k - i])));
        if (tid == 0) nxt[k] = kap;
        P *= 1.0 - (kap.x * kap.x + kap.y * kap.y);
        ok = P > 0.0 && isfinite(P);
        double2* sw = cur;
        cur = nxt;
        nxt = sw;
        __syncthreads();
    }
    if (!ok) {
        if (tid == 0 && atomicCAS(status, 0, LMMSE_ERR_NOT_PD) == 0) status[1] = 0;
        return;
    }
    // x = A^-1 e_0 = [1; p] / P
    const double iP = 1.0 / P;
    for (int i = tid; i < n; i += 64) {
        const double2 v = i == 0 ? make_double2(1.0, 0.0) : cur[i];
        xout[i] = make_double2(v.x * iP, v.y * iP);
    }
}

// Gohberg-Semencul fill of A^-1 from its first column x (y_k = conj(x_{n-1-k})
// the last column): along a diagonal Ainv[i][j] = Ainv[i-1][j-1] +
// (x_i conj(x_j) - y_{i-1} conj(y_{j-1})) / x_0, so for i >= j, d = i - j,
//     Ainv[i][j] = x_d + sum_{s=1..j} (x_{d+s} conj(x_s) - y_{d+s-1} conj(y_{s-1})) / x_0,
// and Ainv[j][i] = conj(Ainv[i][j]).  One thread per entry, column-major.
__global__ __launch_bounds__(256) void gs_fill_kernel(const double2* __restrict__ xg, int n,
                                                      double2* __restrict__ ainv) {
    extern __shared__ double2 xs[];
    for (int t = threadIdx.x; t < n; t += blockDim.x) xs[t] = xg[t];
    __syncthreads();
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * n) return;
    const int i0 = (int)(idx % n), j0 = (int)(idx / n);
    const bool up = i0 < j0;
    const int i = up ? j0 : i0, j = up ? i0 : j0, d = i - j;
    const double ix0 = 1.0 / xs[0].x;
    double vx = 0.0, vy = 0.0;
    for (int s = 1; s <= j; ++s) {
        const double2 t1 = zmulc(xs[d + s], xs[s]);
        // y_{d+s-1} conj(y_{s-1}) = conj(x_{n-d-s}) x_{n-s}
        const double2 t2 = zmulc(xs[n - s], xs[n - d - s]);
        vx += t1.x - t2.x;
        vy += t1.y - t2.y;
    }
    double2 v = make_double2(xs[d].x + vx * ix0, xs[d].y + vy * ix0);
    ainv[idx] = up ? zconj(v) : v;
}

// W_c[i][j] = delta(off_c + i, j) - lam Ainv[off_c + i][j].
__global__ void extract_kernel(const double2* __restrict__ ainv, const int* __restrict__ class_off,
                               double2* __restrict__ w, int n_classes, int B, int n, double lam) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)B * n;
    if (idx >= per * n_classes) return;
    const int c = (int)(idx / per);
    const long long r = idx % per;
    const int i = (int)(r / n), j = (int)(r % n);
    const int row = class_off[c] + i;
    const double2 v = ainv[row + (long long)j * n];
    w[idx] = make_double2((row == j ? 1.0 : 0.0) - lam * v.x, -lam * v.y);
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
                                int n_classes, int B, int Wn, int ngroups, int RT, int rgroups) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int rows = RT * 16;
    const long long total = (long long)n_classes * ngroups * rgroups * 4 * rows;
    if (idx >= total) return;
    const int rr = (int)(idx % rows);
    long long t = idx / rows;
    const int q = (int)(t & 3);
    t >>= 2;
    const int rg = (int)(t % rgroups);
    t /= rgroups;
    const int g = (int)(t % ngroups);
    const int c = (int)(t / ngroups);
    const int r = rg * rows + rr;
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

// Split parts of the real embedding: hi = round(x), lo = round(x - hi) in
// BF16; FP16 stores lo = round(2^11 (x - hi)).
// FP16 banks: the filtering kernel forms 2^11 hi, so every filter entry must
// be below 32 in magnitude; a larger one records LMMSE_ERR_RANGE.
__global__ void pack_split_kernel(const double2* __restrict__ w64, uint16_t* __restrict__ hi,
                                  uint16_t* __restrict__ lo, int n_classes, int B, int Wn, int G16, int RT, int rgroups,
                                  int is_fp16, int* status) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int rows = RT * 16;
    const long long total = (long long)n_classes * G16 * rgroups * 4 * rows * 8;
    if (idx >= total) return;
    const int e = (int)(idx & 7);
    long long t = idx >> 3;
    const int rr = (int)(t % rows);
    t /= rows;
    const int kq = (int)(t & 3);
    t >>= 2;
    const int rg = (int)(t % rgroups);
    t /= rgroups;
    const int g = (int)(t % G16);
    const int c = (int)(t / G16);
    const int r = rg * rows + rr;
    const double x = wreal(w64 + (long long)c * B * Wn, B, Wn, r, 32 * g + 8 * kq + e);
    if (is_fp16) {
        if (!(fabs(x) < 32.0) && atomicCAS(status, 0, LMMSE_ERR_RANGE) == 0) status[1] = -1;
        const _Float16 h = (_Float16)x;
        const _Float16 l = (_Float16)((x - (double)h) * 2048.0);
        hi[idx] = __builtin_bit_cast(uint16_t, h);
        lo[idx] = __builtin_bit_cast(uint16_t, l);
    } else {
        const uint16_t h = f32_to_bf16((float)x);
        const uint16_t l = f32_to_bf16((float)(x - (double)bf16_to_f32(h)));
        hi[idx] = h;
        lo[idx] = l;
    }
}

hipError_t launch_pack_banks(Plan& p, hipStream_t st) {
    const int B = p.d.B, Wn = p.d.Wn;
    {
        const long long total = (long long)fixed_bank_f32_elems(p);
        hipLaunchKernelGGL(pack_f32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                           p.w64, p.wf32, p.n_classes, B, Wn, 2 * p.G16, p.RT, p.rgroups);
    }
    if (p.whi) {
        const long long total = (long long)split_bank_elems(p);
        hipLaunchKernelGGL(pack_split_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                           st, p.w64, p.whi, p.wlo, p.n_classes, B, Wn, p.G16, p.RT,
                           p.rgroups, p.d.precision == LMMSE_FP16X3 ? 1 : 0, p.status);
    }
    return hipGetLastError();
}

hipError_t launch_fixed_design(Plan& p, double tau, double sigma2, hipStream_t st) {
    const int n = p.d.Wn;
    const double lam = sigma2 / p.d.K;
    hipLaunchKernelGGL(rd_kernel, dim3(n), dim3(64), 0, st, p.rd, n, p.d.rsource, p.d.L, tau,
                       p.d.taps, p.d.N_fft);
    hipLaunchKernelGGL(toeplitz_inverse_kernel, dim3(1), dim3(64), (size_t)3 * n * sizeof(double2),
                       st, p.rd, n, lam, p.rd + 2 * n, p.status);
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(gs_fill_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256),
                       (size_t)n * sizeof(double2), st, p.rd + 2 * n, n, p.ainv);
    const long long tot = (long long)p.n_classes * p.d.B * n;
    hipLaunchKernelGGL(extract_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       p.ainv, p.d_class_off, p.w64, p.n_classes, p.d.B, n, lam);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_pack_banks(p, st);
}

}  // namespace lmmse
