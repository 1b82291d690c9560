// Backward of the sample-covariance estimator.  Per (slot s, user k, block b)
// let X = h_ls[s, :, k, I_b]^T (Wn x M), G = g[s, :, k, O_b]^T (B x M),
// A = X X^H / M + lam I and W = R_OI A^-1 (eq. 13 on the window).  With the
// gradient convention dL = Re sum conj(grad z) dz:
//     dW   = G X^H                           (B x Wn)
//     Z    = dW A^-1                         (B x Wn)
//     Gam  = -W^H Z,  then Gam[off + o, :] += Z[o, :]   (gradient of R, Wn x Wn)
//     dX   = W^H G + S X,  S = (Gam + Gam^H) / M   (R depends on X: dR = (dX X^H + X dX^H) / M)
//     dlam = Re tr(-W^H Z), summed over all windows.
// The window gradients are written per window and combined afterwards in a
// fixed order (overlapping windows add), so the result does not depend on
// scheduling.
//
// The window products are batched complex GEMMs with FP64 accumulation
// (zgemm.h; the solve-side products Z and Gam need FP64, the others reuse the
// same kernel).  Each operand is a strided view into h_ls, g or a per-window
// buffer.
#include <algorithm>

#include "zgemm.h"

namespace lmmse {

// Per window: dlam partial = Re tr(Gam) (Gam = -W^H Z as computed so far),
// and S = (Gam' + Gam'^H) / M in place of Gam, where Gam' is Gam with Z's rows
// added to rows off .. off + B - 1.  One pass over 32 x 32 tile pairs (I, J),
// I >= J: both tiles are loaded with their Z rows (every load issued, element
// 0 standing in outside, so that a tile's loads are in flight together) and
// staged in LDS, so that every global access walks a row; the diagonal of
// Gam is kept aside before Z is added, and summed in the order of a
// 256-thread tree (Wn <= kMaxSampleWindowLarge = 256).
__global__ __launch_bounds__(256) void gamma_rows_kernel(double2* gam, const double2* z,
                                                         const int* offsets, double* dlam_w, int B,
                                                         int Wn, int nb, double invM) {
    __shared__ double red[256];
    __shared__ double dg[kMaxSampleWindowLarge];
    __shared__ double2 t1[32][33], t2[32][33];
    const long long mat = blockIdx.x;
    const int tid = threadIdx.x, off = offsets[mat % nb];
    double2* gm = gam + mat * Wn * Wn;
    const double2* zm = z + mat * B * Wn;
    const int nt = (Wn + 31) / 32;
    for (int I = 0; I < nt; ++I)
        for (int J = 0; J <= I; ++J) {
            double2 a1[4], a2[4], z1[4], z2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + 256 * u, r = e >> 5, c = e & 31;
                const int i1 = 32 * I + r, j1 = 32 * J + c, i2 = 32 * J + r, j2 = 32 * I + c;
                const bool ok1 = i1 < Wn && j1 < Wn, ok2 = i2 < Wn && j2 < Wn;
                const bool in1 = ok1 && i1 >= off && i1 < off + B, in2 = ok2 && i2 >= off && i2 < off + B;
                a1[u] = gm[ok1 ? (long long)i1 * Wn + j1 : 0];
                a2[u] = gm[ok2 ? (long long)i2 * Wn + j2 : 0];
                z1[u] = zm[in1 ? (long long)(i1 - off) * Wn + j1 : 0];
                z2[u] = zm[in2 ? (long long)(i2 - off) * Wn + j2 : 0];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + 256 * u, r = e >> 5, c = e & 31;
                const int i1 = 32 * I + r, j1 = 32 * J + c, i2 = 32 * J + r, j2 = 32 * I + c;
                const bool ok1 = i1 < Wn && j1 < Wn, ok2 = i2 < Wn && j2 < Wn;
                const bool in1 = ok1 && i1 >= off && i1 < off + B, in2 = ok2 && i2 >= off && i2 < off + B;
                if (I == J && r == c && ok1) dg[i1] = a1[u].x;
                t1[r][c] = !ok1 ? make_double2(0.0, 0.0)
                                : in1 ? make_double2(a1[u].x + z1[u].x, a1[u].y + z1[u].y) : a1[u];
                t2[r][c] = !ok2 ? make_double2(0.0, 0.0)
                                : in2 ? make_double2(a2[u].x + z2[u].x, a2[u].y + z2[u].y) : a2[u];
            }
            __syncthreads();
            for (int e = tid; e < 1024; e += 256) {
                const int r = e >> 5, c = e & 31;
                const int i1 = 32 * I + r, j1 = 32 * J + c, i2 = 32 * J + r, j2 = 32 * I + c;
                // S[i1][j1] = (Gam'[i1][j1] + conj(Gam'[j1][i1])) / M, Gam'[j1][i1] = t2[c][r]
                if (i1 < Wn && j1 < Wn) {
                    const double2 a = t1[r][c], b = t2[c][r];
                    gm[(long long)i1 * Wn + j1] = make_double2((a.x + b.x) * invM, (a.y - b.y) * invM);
                }
                if (I != J && i2 < Wn && j2 < Wn) {
                    const double2 a = t2[r][c], b = t1[c][r];
                    gm[(long long)i2 * Wn + j2] = make_double2((a.x + b.x) * invM, (a.y - b.y) * invM);
                }
            }
            __syncthreads();
        }
    double tr = 0.0;
    for (int i = tid; i < Wn; i += 256) tr += dg[i];
    red[tid] = tr;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) dlam_w[mat] = red[0];
}

// dhls[s, m, k, n] = sum over the windows b that hold n, in increasing b, of
// dxw[(s, k, b)][m][n - start_b].
__global__ __launch_bounds__(256) void combine_windows_kernel(const float2* dxw, const int* starts,
                                                              float2* dhls, int M, int K, int N,
                                                              int B, int Wn, int nb,
                                                              long long total) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int n = (int)(e % N);
    long long r = e / N;
    const int k = (int)(r % K);
    r /= K;
    const int m = (int)(r % M);
    const long long s = r / M;
    // a window that holds n starts within ceil(Wn / B) + 1 blocks of n's block
    const int bc = n / B, halo_blocks = (Wn + B - 1) / B + 1;
    const int blo = max(0, bc - halo_blocks), bhi = min(nb - 1, bc + halo_blocks);
    // candidates four at a time, every load issued (a window that does not
    // hold n reads its element 0 and adds nothing), so that a group's loads
    // are in flight together; the sum runs in window order
    float sx = 0.f, sy = 0.f;
    for (int b0 = blo; b0 <= bhi; b0 += 4) {
        float2 v[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = min(b0 + u, bhi), j = n - starts[b];
            ok[u] = b0 + u <= bhi && j >= 0 && j < Wn;
            const long long mat = (s * K + k) * nb + b;
            v[u] = dxw[(mat * M + m) * Wn + (ok[u] ? j : 0)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (ok[u]) {
                sx += v[u].x;
                sy += v[u].y;
            }
    }
    dhls[e] = make_float2(sx, sy);
}

// Fixed-order sum of the per-window dlam partials into out[1]; out[0] (the
// delay-spread gradient of the fixed design) is NaN here.
__global__ __launch_bounds__(256) void dlam_sum_kernel(const double* dlam_w, long long nmat,
                                                       double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (long long i = threadIdx.x; i < nmat; i += 256) s += dlam_w[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = __builtin_nan("");
        out[1] = red[0];
    }
}

namespace {
size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Per-window buffers of one chunk of slots.
struct SbLayout {
    size_t ainv, w64, dw, z, dxw, panel, total;
};

SbLayout sb_layout(const lmmse_plan_desc& d, int slots) {
    const long long nmat = (long long)slots * d.K * (d.N / d.B);
    SbLayout L{};
    size_t o = 0;
    L.ainv = o;
    o += up256((size_t)nmat * d.Wn * d.Wn * sizeof(double2));
    L.w64 = o;
    o += up256((size_t)nmat * d.B * d.Wn * sizeof(double2));
    L.dw = o;
    o += up256((size_t)nmat * d.B * d.Wn * sizeof(double2));
    L.z = o;
    o += up256((size_t)nmat * d.B * d.Wn * sizeof(double2));
    L.dxw = o;
    o += up256((size_t)nmat * d.M * d.Wn * sizeof(float2));
    L.panel = o;   // panel operands of the workspace-resident design (wide windows)
    if (d.Wn > kMaxSampleWindowReg) o += up256(sweep_scratch_bytes(d.Wn, nmat));
    L.total = o;
    return L;
}

// Slots per chunk: as many as fit in the forward estimate's workspace (at
// least one), so that the backward needs little more memory than the forward.
int sb_chunk(const lmmse_plan_desc& d, int slots) {
    if (slots <= 0) return 0;
    const size_t fwd = sample_workspace_bytes(d, slots), per = sb_layout(d, 1).total;
    const size_t c = per ? fwd / per : (size_t)slots;
    return (int)std::min<size_t>(std::max<size_t>(c, 1), (size_t)slots);
}

size_t dlam_bytes(const lmmse_plan_desc& d, int slots) {
    return up256((size_t)slots * d.K * (d.N / d.B) * sizeof(double));
}

ZView hview(const lmmse_plan_desc& d, const float2* p, const int* tab, long long s_blk, int conj,
            bool transposed) {
    // element (row, col) = (window or block row, antenna), or its transpose
    ZView v{};
    v.p = p;
    const long long ms = (long long)d.K * d.N;
    v.rs = transposed ? ms : 1;
    v.cs = transposed ? 1 : ms;
    v.s_slot = (long long)d.M * d.K * d.N;
    v.s_user = d.N;
    v.s_blk = s_blk;
    v.blk_tab = tab;
    v.conj = conj;
    return v;
}

ZView wview(const void* p, const lmmse_plan_desc& d, int rows, int cols, bool conj_t) {
    // per-window buffer [mat][rows][cols]; conj_t: the conjugate transpose
    ZView v{};
    v.p = p;
    const long long per = (long long)rows * cols;
    v.rs = conj_t ? 1 : cols;
    v.cs = conj_t ? cols : 1;
    v.s_blk = per;
    v.s_user = per * (d.N / d.B);
    v.s_slot = v.s_user * d.K;
    v.blk_tab = nullptr;
    v.conj = conj_t ? 1 : 0;
    return v;
}
}  // namespace

size_t sample_backward_workspace_bytes(const lmmse_plan_desc& d, int slots) {
    if (slots <= 0) return 0;
    return dlam_bytes(d, slots) + sb_layout(d, sb_chunk(d, slots)).total;
}

hipError_t launch_backward_sample(Plan& p, int slots, const float2* hls, const float2* g,
                                  float2* dhls, double lam, bool want_sigma, void* ws,
                                  hipStream_t st, const double2* kept_w64, const double2* kept_ainv) {
    const lmmse_plan_desc& d = p.d;
    if (d.Wn > kMaxSampleWindowLarge) return hipErrorInvalidValue;   // gamma_rows_kernel's diagonal
    if ((long long)slots * d.K * p.nb == 0) return hipSuccess;
    const int chunk = sb_chunk(d, slots);
    const SbLayout L = sb_layout(d, chunk);
    char* w = (char*)ws;
    double* dlam = (double*)w;
    w += dlam_bytes(d, slots);
    double2* ainv = (double2*)(w + L.ainv);   // A^-1, then Gam
    double2* w64 = (double2*)(w + L.w64);
    double2* dw = (double2*)(w + L.dw);
    double2* z = (double2*)(w + L.z);
    float2* dxw = (float2*)(w + L.dxw);
    const int B = d.B, Wn = d.Wn, M = d.M;
    const long long per_slot = (long long)M * d.K * d.N;
    hipError_t e;

    for (int s0 = 0; s0 < slots; s0 += chunk) {
        const int ns = std::min(chunk, slots - s0);
        const long long nmat = (long long)ns * d.K * p.nb, mat0 = (long long)s0 * d.K * p.nb;
        const float2* hc = hls + s0 * per_slot;
        const float2* gc = g + s0 * per_slot;

        // the chunk's W rows and A^-1: kept by the forward, or designed again
        // into the workspace; Gam then goes to the workspace's A^-1 area
        const double2* wsrc = w64;
        const double2* asrc = ainv;
        if (kept_ainv) {
            wsrc = kept_w64 + mat0 * B * Wn;
            asrc = kept_ainv + mat0 * Wn * Wn;
        } else {
            e = launch_sample_inverse(p, nmat, mat0, hc, lam, w64, ainv, (double2*)(w + L.panel), st);
            if (e != hipSuccess) return e;
        }

        ZGemmArgs ga{};
        ga.K = d.K;
        ga.nb = p.nb;
        // dW = G X^H
        ga.A = hview(d, gc, nullptr, B, 0, false);
        ga.B = hview(d, hc, p.d_starts, 1, 1, true);
        ga.C = wview(dw, d, B, Wn, false);
        ga.m = B;
        ga.n = Wn;
        ga.kd = M;
        ga.alpha = 1.0;
        ga.beta = 0;
        if ((e = zgemm<float2, float2, double2>(ga, nmat, st)) != hipSuccess) return e;
        // Z = dW A^-1
        ga.A = wview(dw, d, B, Wn, false);
        ga.B = wview(asrc, d, Wn, Wn, false);
        ga.C = wview(z, d, B, Wn, false);
        ga.kd = Wn;
        if ((e = zgemm<double2, double2, double2>(ga, nmat, st)) != hipSuccess) return e;
        // Gam = -W^H Z (over the workspace's A^-1, which is no longer needed)
        ga.A = wview(wsrc, d, B, Wn, true);
        ga.B = wview(z, d, B, Wn, false);
        ga.C = wview(ainv, d, Wn, Wn, false);
        ga.m = Wn;
        ga.n = Wn;
        ga.kd = B;
        ga.alpha = -1.0;
        if ((e = zgemm<double2, double2, double2>(ga, nmat, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(gamma_rows_kernel, dim3((unsigned)nmat), dim3(256), 0, st, ainv, z,
                           p.d_offsets, dlam + mat0, B, Wn, p.nb, 1.0 / M);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // per-window dX, stored [mat][m][j]: W^H G + S X, in FP32 arithmetic
        // (the result is the FP32 gradient; FP64 stays where the solve is)
        ZView cx{};
        cx.p = dxw;
        cx.rs = 1;
        cx.cs = Wn;
        cx.s_blk = (long long)M * Wn;
        cx.s_user = cx.s_blk * p.nb;
        cx.s_slot = cx.s_user * d.K;
        ga.A = wview(wsrc, d, B, Wn, true);
        ga.B = hview(d, gc, nullptr, B, 0, false);
        ga.C = cx;
        ga.m = Wn;
        ga.n = M;
        ga.kd = B;
        ga.alpha = 1.0;
        ga.beta = 0;
        if ((e = zgemm<double2, float2, float2, float>(ga, nmat, st)) != hipSuccess) return e;
        ga.A = wview(ainv, d, Wn, Wn, false);
        ga.B = hview(d, hc, p.d_starts, 1, 0, false);
        ga.kd = Wn;
        ga.beta = 1;
        if ((e = zgemm<double2, float2, float2, float>(ga, nmat, st)) != hipSuccess) return e;

        const long long total = ns * per_slot;
        hipLaunchKernelGGL(combine_windows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256),
                           0, st, dxw, p.d_starts, dhls + s0 * per_slot, M, d.K, d.N, B, Wn, p.nb,
                           total);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (want_sigma) {
        hipLaunchKernelGGL(dlam_sum_kernel, dim3(1), dim3(256), 0, st, dlam,
                           (long long)slots * d.K * p.nb, p.dscal);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lmmse
