// MMSE MIMO detection (Sec. IV-A, MMSE MIMO detector, eq. 20-22): per (slot s, data
// subcarrier n), with H = h_hat[s, :, :, n] (M x K) and Y = y[s, :, :, n]
// (M x T), the detected symbols solve
//     (H^H H + sigma2 I) X = H^H Y                                  (eq. 22)
// by a Cholesky factorisation A = L L^H and two triangular solves per data
// symbol, in FP32 (the paper's LAPACKE_cposv is the single-precision
// complex routine).
//
// One workgroup per (slot, 16 consecutive subcarriers).  Antennas are
// streamed through LDS 8 at a time (each (antenna, user) row of 16
// subcarriers is one 128-byte load); thread (l, i) accumulates row i of
// [H^H H | H^H Y] for subcarrier l in registers.  The rows go to LDS (over the staging area, after the last
// antenna), A is factored in place column by column (each row by its own
// thread), and one thread per (subcarrier, data symbol) solves and writes
// its K symbols.
#include <algorithm>

#include "internal.h"

namespace lmmse {

constexpr int dNB = 16;   // subcarriers per workgroup
constexpr int dMC = 8;    // antennas per LDS stage
constexpr int dMaxK = 16, dMaxT = 16;

__device__ __forceinline__ float2 cmul_conj_a(float2 a, float2 b) {   // conj(a) b
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// KTC = K + T rounded up to a multiple of 4 (rows K + T .. KTC - 1 of the
// staged [H | Y] are zero), so that the staging and the Gram loops have
// compile-time trip counts: every thread issues all of its loads of a stage
// before storing any, and the accumulation runs without branches.
template <int KTC>
__global__ __launch_bounds__(256) void mmse_detect_kernel(const float2* h, const float2* y, float2* x,
                                                          int M, int K, int T, int N, float sigma2,
                                                          int nblk) {
    static_assert(KTC % 4 == 0 && KTC <= dMaxK + dMaxT, "row count");
    extern __shared__ float2 sm[];
    const int KT = K + T;
    float2* Hs = sm;                         // [dMC][KTC][dNB]: rows q < K of H, then Y, then zeros
    float2* Gs = sm;                         // [dNB][K][KT], after the antenna loop
    const int tid = threadIdx.x, l = tid & (dNB - 1), i = tid / dNB;
    const long long s = blockIdx.x / nblk;
    const int n0 = (int)(blockIdx.x % nblk) * dNB;
    const float2* hs = h + s * (long long)M * K * N;
    const float2* ys = y + s * (long long)M * T * N;
    const bool nlive = n0 + l < N;

    float2 acc[KTC];
#pragma unroll
    for (int c = 0; c < KTC; ++c) acc[c] = make_float2(0.f, 0.f);

    // thread (l, i) stages rows q = i and i + 16 (those below KTC) of every
    // antenna of a stage: one base pointer and stride per row
    const float2* qp[2];
    long long qs[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const int q = i + 16 * w;
        qp[w] = (q < K ? hs + (long long)q * N : ys + (long long)(q - K) * N) + n0 + l;
        qs[w] = q < K ? (long long)K * N : (long long)T * N;
    }
    // the loads of stage m0 + dMC are issued before the Gram updates of
    // stage m0 and stored to LDS after them
    float2 v[2][dMC];
    auto load_stage = [&](int m0) {
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int q = i + 16 * w;
#pragma unroll
            for (int mm = 0; mm < dMC; ++mm) {
                v[w][mm] = make_float2(0.f, 0.f);
                if (q < KTC && nlive && m0 + mm < M && q < KT) v[w][mm] = qp[w][(m0 + mm) * qs[w]];
            }
        }
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int q = i + 16 * w;
            if (q < KTC) {
#pragma unroll
                for (int mm = 0; mm < dMC; ++mm) Hs[(mm * KTC + q) * dNB + l] = v[w][mm];
            }
        }
    };
    load_stage(0);
    store_stage();
    __syncthreads();
    for (int m0 = 0; m0 < M; m0 += dMC) {
        const bool more = m0 + dMC < M;
        if (more) load_stage(m0 + dMC);
        if (i < K) {
#pragma unroll 2
            for (int mm = 0; mm < dMC; ++mm) {
                const float2* hm = Hs + mm * KTC * dNB + l;
                const float2 hi = hm[i * dNB];
#pragma unroll
                for (int c = 0; c < KTC; ++c) {
                    const float2 p = cmul_conj_a(hi, hm[c * dNB]);
                    acc[c].x += p.x;
                    acc[c].y += p.y;
                }
            }
        }
        __syncthreads();
        if (more) store_stage();
        __syncthreads();
    }
    if (i < K) {
        float2* g = Gs + (l * K + i) * KT;
#pragma unroll
        for (int c = 0; c < KTC; ++c)
            if (c < KT) g[c] = acc[c];
        g[i].x += sigma2;
    }
    __syncthreads();
    float2* G = Gs + l * K * KT;   // this subcarrier's [A | B]
    // A = L L^H in place, column by column: the diagonal entry by its row's
    // thread, then every row below it by its own thread (L_jj real)
    for (int j = 0; j < K; ++j) {
        if (i == j) {
            float d = G[j * KT + j].x;
            for (int q = 0; q < j; ++q) {
                const float2 v = G[j * KT + q];
                d -= v.x * v.x + v.y * v.y;
            }
            G[j * KT + j] = make_float2(d > 0.f ? sqrtf(d) : __builtin_nanf(""), 0.f);
        }
        __syncthreads();
        if (i > j && i < K) {
            float2 v = G[i * KT + j];
            for (int q = 0; q < j; ++q) {   // v -= L_iq conj(L_jq)
                const float2 a = G[i * KT + q], b = G[j * KT + q];
                v.x -= a.x * b.x + a.y * b.y;
                v.y -= a.y * b.x - a.x * b.y;
            }
            const float inv = 1.0f / G[j * KT + j].x;
            G[i * KT + j] = make_float2(v.x * inv, v.y * inv);
        }
        __syncthreads();
    }
    const int t = i;
    if (t < T && n0 + l < N) {
        float2 z[dMaxK];
        // L z = b (every index compile-time after unrolling: z stays in registers)
#pragma unroll
        for (int r = 0; r < dMaxK; ++r) {
            z[r] = make_float2(0.f, 0.f);
            if (r < K) {
                float2 v = G[r * KT + K + t];
#pragma unroll
                for (int q = 0; q < r; ++q) {
                    const float2 a = G[r * KT + q];
                    v.x -= a.x * z[q].x - a.y * z[q].y;
                    v.y -= a.x * z[q].y + a.y * z[q].x;
                }
                const float inv = 1.0f / G[r * KT + r].x;
                z[r] = make_float2(v.x * inv, v.y * inv);
            }
        }
        // L^H x = z
#pragma unroll
        for (int r = dMaxK - 1; r >= 0; --r) {
            if (r < K) {
                float2 v = z[r];
#pragma unroll
                for (int q = r + 1; q < dMaxK; ++q) {   // v -= conj(L_qr) x_q
                    if (q < K) {
                        const float2 a = G[q * KT + r];
                        v.x -= a.x * z[q].x + a.y * z[q].y;
                        v.y -= a.x * z[q].y - a.y * z[q].x;
                    }
                }
                const float inv = 1.0f / G[r * KT + r].x;
                z[r] = make_float2(v.x * inv, v.y * inv);
            }
        }
        float2* xs = x + (s * T + t) * (long long)K * N + n0 + l;
#pragma unroll
        for (int k = 0; k < dMaxK; ++k)
            if (k < K) xs[(long long)k * N] = z[k];
    }
}

}  // namespace lmmse

extern "C" int lmmse_mmse_detect(int slots, int M, int K, int T, int N, const void* h_hat,
                                 const void* y_data, double sigma2, void* x_out, void* stream) {
    if (slots < 0 || M < 1 || K < 1 || T < 1 || N < 1) return LMMSE_ERR_INVALID_ARG;
    if (!(sigma2 > 0.0) || !(sigma2 < 1e30)) return LMMSE_ERR_INVALID_ARG;
    if (K > lmmse::dMaxK || T > lmmse::dMaxT) return LMMSE_ERR_UNSUPPORTED;
    if (slots == 0) return LMMSE_OK;
    if (!h_hat || !y_data || !x_out) return LMMSE_ERR_INVALID_ARG;
    const int nblk = (N + lmmse::dNB - 1) / lmmse::dNB;
    const int ktc = (K + T + 3) & ~3;
    const size_t shm = std::max((size_t)lmmse::dMC * ktc * lmmse::dNB,
                                (size_t)lmmse::dNB * K * (K + T)) * sizeof(float2);
    const dim3 grid((unsigned)((long long)slots * nblk)), block(256);
    const hipStream_t st = (hipStream_t)stream;
    const float2 *hp = (const float2*)h_hat, *yp = (const float2*)y_data;
    float2* xp = (float2*)x_out;
    switch (ktc) {
#define LMMSE_DK(C)                                                                              \
    case C:                                                                                      \
        hipLaunchKernelGGL(lmmse::mmse_detect_kernel<C>, grid, block, shm, st, hp, yp, xp, M, K, \
                           T, N, (float)sigma2, nblk);                                           \
        break;
        LMMSE_DK(4) LMMSE_DK(8) LMMSE_DK(12) LMMSE_DK(16) LMMSE_DK(20) LMMSE_DK(24) LMMSE_DK(28)
        LMMSE_DK(32)
#undef LMMSE_DK
        default:
            return LMMSE_ERR_UNSUPPORTED;
    }
    return hipGetLastError() == hipSuccess ? LMMSE_OK : LMMSE_ERR_HIP;
}
