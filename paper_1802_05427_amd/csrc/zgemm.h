// Batched complex GEMM over strided operand views (used by the
// sample-covariance design for windows too wide for the register-resident
// sweep, and by its backward) on the matrix cores: FP64, or FP32 for
// products that only need FP32 accuracy.
#pragma once

#include "internal.h"

namespace lmmse {

// Matrix view: element (r, c) of batch (s, k, b) sits at
//   p + s*s_slot + k*s_user + (blk_tab ? blk_tab[b] : b)*s_blk + r*rs + c*cs,
// conjugated when conj is set.
struct ZView {
    const void* p;
    long long rs, cs, s_slot, s_user, s_blk;
    const int* blk_tab;
    int conj;
};

struct ZGemmArgs {
    ZView A, B, C;       // C = alpha A B (+ C when beta); C.p is written
    int m, n, kd;        // C is m x n, the contraction has kd terms
    int K, nb;           // batch index = (s * K + k) * nb + b
    int tiles_m, tiles_n;
    double alpha;
    int beta;
    int herm;            // C and the update Hermitian (square): compute the lower
                         // tiles, mirror them
    int skip_tile = -1;  // when >= 0: the 64-row tile row of that index (and, for a
                         // Hermitian product, the tile column) is left out: the
                         // caller knows the product vanishes there or is not read
    ZView T;             // when tcopy is set (not with herm), element (r, c) of the
    int tcopy;           // result is also written conjugated at T's element (c, r)
};

constexpr int zT = 64;    // output tile edge
constexpr int zKC = 16;   // contraction chunk

__device__ __forceinline__ long long zbase(const ZView& v, long long bat, int K, int nb) {
    const int b = (int)(bat % nb);
    const long long sk = bat / nb;
    const int k = (int)(sk % K);
    const long long s = sk / K;
    return s * v.s_slot + k * v.s_user + (long long)(v.blk_tab ? v.blk_tab[b] : b) * v.s_blk;
}

// Complex accumulator / LDS element of a precision: FP64 (double2) or FP32 (float2).
template <typename R>
struct Cx;
template <>
struct Cx<double> {
    using T = double2;
    __device__ static T make(double x, double y) { return make_double2(x, y); }
};
template <>
struct Cx<float> {
    using T = float2;
    __device__ static T make(double x, double y) { return make_float2((float)x, (float)y); }
};

// The product on the matrix cores: a workgroup computes one 64 x 64 output
// tile, staging 16-term chunks of A and B through LDS (the next chunk's loads
// in flight during the current chunk's MFMAs); each wave owns a 32 x 32
// quarter as 2 x 2 MFMA tiles (one sub-tile each in a tile with a single
// live row or column of them), real and imaginary parts in separate
// accumulators (4 real products per complex one).  Operand lane (i, k) =
// (lane % 16, lane / 16).  R is the arithmetic precision: double
// (v_mfma_f64_16x16x4f64, FP64 products and sums) or float
// (v_mfma_f32_16x16x4f32, for products whose result only needs FP32
// accuracy).
typedef double zd4 __attribute__((ext_vector_type(4)));
typedef float zf4 __attribute__((ext_vector_type(4)));

template <typename R>
struct ZMma;
template <>
struct ZMma<double> {
    using V = zd4;
    __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // accumulator element v of lane l: row 4 v + l / 16, column l % 16
    __device__ static int row(int v, int lk) { return 4 * v + lk; }
};
template <>
struct ZMma<float> {
    using V = zf4;
    __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // accumulator element v of lane l: row 4 (l / 16) + v, column l % 16
    __device__ static int row(int v, int lk) { return 4 * lk + v; }
};

// Workgroup id -> tile index such that each of the 8 XCDs (which take
// workgroups round-robin) gets a contiguous range of tiles: the output tiles
// of one batch entry, which read the same operand rows and columns, then run
// side by side under one L2 instead of spread over all eight.
__device__ __forceinline__ long long zgemm_tile_order(long long id, long long total) {
    constexpr long long NX = 8;
    const long long q = total / NX, r = total % NX, x = id % NX, k = id / NX;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Bounded to three waves per SIMD (at most 168 registers per lane): two
// waves per SIMD leave the matrix cores idle while a workgroup stages.
template <typename TA, typename TB, typename TC, typename R>
__global__ __launch_bounds__(256, 3) void zgemm_mfma_kernel(ZGemmArgs g) {
    using CT = typename Cx<R>::T;
    using ZM = ZMma<R>;
    __shared__ CT As[zKC][zT];
    __shared__ CT Bs[zKC][zT];
    const int tid = threadIdx.x;
    long long t = zgemm_tile_order(blockIdx.x, gridDim.x);
    int tm, tn;
    long long bat;
    if (g.herm) {
        const int per = g.tiles_m * (g.tiles_m + 1) / 2;
        int q = (int)(t % per);
        bat = t / per;
        tm = 0;
        while (q > tm) {
            q -= tm + 1;
            ++tm;
        }
        tn = q;
    } else {
        tn = (int)(t % g.tiles_n);
        t /= g.tiles_n;
        tm = (int)(t % g.tiles_m);
        bat = t / g.tiles_m;
    }
    if (g.skip_tile >= 0) {   // tiles_m (and, Hermitian, the square) count the others
        tm += tm >= g.skip_tile ? 1 : 0;
        if (g.herm) tn += tn >= g.skip_tile ? 1 : 0;
    }
    const int r0 = tm * zT, c0 = tn * zT;
    const long long abase = zbase(g.A, bat, g.K, g.nb);
    const long long bbase = zbase(g.B, bat, g.K, g.nb);
    const long long cbase = zbase(g.C, bat, g.K, g.nb);
    const bool a_rowfast = g.A.rs == 1, b_colfast = g.B.cs == 1;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    // A tile whose rows end within its first 16 has one live row of
    // sub-tiles: wave w takes sub-tile (0, w) there, not a 2 x 2 block, so
    // that all four waves share the work; likewise sub-tile (w, 0) of a tile
    // whose columns end within its first 16.
    const bool ragged = r0 + 16 >= g.m;
    const bool cragged = !ragged && c0 + 16 >= g.n;
    const int wr = ragged ? 0 : (wave >> 1) * 32;
    const int wc = ragged ? (wave >> 1) * 32 : cragged ? 0 : (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;

    typename ZM::V cre[2][2], cim[2][2];
    // 16 x 16 sub-tiles this wave computes (wave-uniform): those with rows and
    // columns in range and, on a diagonal tile of a Hermitian product, on or
    // below the diagonal (the upper ones are written as mirrors)
    bool live[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            cre[i][j] = typename ZM::V{0, 0, 0, 0};
            cim[i][j] = typename ZM::V{0, 0, 0, 0};
            const int ri = wr + 16 * i, cj = wc + 16 * j;
            live[i][j] = r0 + ri < g.m && c0 + cj < g.n && !(g.herm && tm == tn && ri < cj) &&
                         (!ragged || (i == 0 && j == (wave & 1))) &&
                         (!cragged || (j == 0 && i == (wave & 1)));
        }

    // Every thread issues all eight loads of a chunk unconditionally (an
    // element outside the operand reads the batch's element (0, 0) instead
    // and is zeroed after the load): loads under a branch would each be
    // waited for before the next is issued.
    TA ra[4];
    TB rb[4];
    bool oka[4], okb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            const int r = a_rowfast ? (e & 63) : (e >> 4), ka = a_rowfast ? (e >> 6) : (e & 15);
            const int c = b_colfast ? (e & 63) : (e >> 4), kb = b_colfast ? (e >> 6) : (e & 15);
            oka[u] = r0 + r < g.m && k0 + ka < g.kd;
            okb[u] = c0 + c < g.n && k0 + kb < g.kd;
            ra[u] = reinterpret_cast<const TA*>(g.A.p)[oka[u] ? abase + (r0 + r) * g.A.rs + (k0 + ka) * g.A.cs
                                                               : abase];
            rb[u] = reinterpret_cast<const TB*>(g.B.p)[okb[u] ? bbase + (k0 + kb) * g.B.rs + (c0 + c) * g.B.cs
                                                               : bbase];
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < g.kd; k0 += zKC) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            const int r = a_rowfast ? (e & 63) : (e >> 4), ka = a_rowfast ? (e >> 6) : (e & 15);
            const int c = b_colfast ? (e & 63) : (e >> 4), kb = b_colfast ? (e >> 6) : (e & 15);
            As[ka][r] = oka[u] ? Cx<R>::make((double)ra[u].x, g.A.conj ? -(double)ra[u].y : (double)ra[u].y)
                               : Cx<R>::make(0.0, 0.0);
            Bs[kb][c] = okb[u] ? Cx<R>::make((double)rb[u].x, g.B.conj ? -(double)rb[u].y : (double)rb[u].y)
                               : Cx<R>::make(0.0, 0.0);
        }
        __syncthreads();
        if (k0 + zKC < g.kd) fetch(k0 + zKC);
#pragma unroll
        for (int ks = 0; ks < zKC / 4; ++ks) {
            const int kk = 4 * ks + lk;
            CT a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kk][wr + 16 * i + li];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kk][wc + 16 * j + li];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if (!live[i][j]) continue;
                    cre[i][j] = ZM::mma(a[i].x, b[j].x, cre[i][j]);
                    cre[i][j] = ZM::mma(-a[i].y, b[j].y, cre[i][j]);
                    cim[i][j] = ZM::mma(a[i].x, b[j].y, cim[i][j]);
                    cim[i][j] = ZM::mma(a[i].y, b[j].x, cim[i][j]);
                }
        }
        __syncthreads();
    }
    TC* cp = reinterpret_cast<TC*>(const_cast<void*>(g.C.p));
    // When accumulating, the old values of C of a row of sub-tiles are read
    // before its first store (unconditional reads, element (0, 0) standing in
    // for those outside), so that the reads are in flight together.  Only
    // elements this thread writes itself are read: the mirrored ones are
    // never read.
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        TC old[2][4];
        if (g.beta) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + wr + 16 * i + ZM::row(v, lk), c = c0 + wc + 16 * j + li;
                    const bool ok = live[i][j] && r < g.m && c < g.n;
                    old[j][v] = cp[ok ? cbase + r * g.C.rs + c * g.C.cs : cbase];
                }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (!live[i][j]) continue;
                const int r = r0 + wr + 16 * i + ZM::row(v, lk), c = c0 + wc + 16 * j + li;
                if (r >= g.m || c >= g.n) continue;
                // mirrors: every sub-tile off the diagonal of a Hermitian product
                const bool mirror = g.herm && (tm != tn || wr + 16 * i > wc + 16 * j);
                const long long o = cbase + r * g.C.rs + c * g.C.cs;
                double x = g.alpha * cre[i][j][v], y = g.alpha * cim[i][j][v];
                if (g.beta) {
                    x += (double)old[j][v].x;
                    y += (double)old[j][v].y;
                }
                if constexpr (sizeof(TC) == sizeof(double2))
                    cp[o] = make_double2(x, y);
                else
                    cp[o] = make_float2((float)x, (float)y);
                if (g.tcopy) {
                    const long long ot = zbase(g.T, bat, g.K, g.nb) + c * g.T.rs + r * g.T.cs;
                    TC* tp = reinterpret_cast<TC*>(const_cast<void*>(g.T.p));
                    if constexpr (sizeof(TC) == sizeof(double2))
                        tp[ot] = make_double2(x, -y);
                    else
                        tp[ot] = make_float2((float)x, (float)-y);
                }
                if (mirror) {
                    const long long om = cbase + c * g.C.rs + r * g.C.cs;
                    if constexpr (sizeof(TC) == sizeof(double2))
                        cp[om] = make_double2(x, -y);
                    else
                        cp[om] = make_float2((float)x, (float)-y);
                }
            }
    }
}

template <typename TA, typename TB, typename TC, typename R = double>
inline hipError_t zgemm(ZGemmArgs g, long long nbat, hipStream_t st) {
    g.tiles_m = (g.m + zT - 1) / zT;
    g.tiles_n = (g.n + zT - 1) / zT;
    if (g.herm && (g.m != g.n || g.tcopy)) return hipErrorInvalidValue;
    if (g.skip_tile >= g.tiles_m) return hipErrorInvalidValue;
    if (g.skip_tile >= 0) --g.tiles_m;   // the kernel maps the remaining tile rows past it
    // the kernel reads element (0, 0) of every batch's A and B
    if (g.kd < 1) return hipErrorInvalidValue;
    const long long blocks =
        nbat * (g.herm ? (long long)g.tiles_m * (g.tiles_m + 1) / 2 : (long long)g.tiles_m * g.tiles_n);
    if (blocks == 0) return hipSuccess;
    if (blocks > (long long)(0xFFFFFFFFu / 256)) return hipErrorInvalidValue;   // work-items < 2^32
    hipLaunchKernelGGL((zgemm_mfma_kernel<TA, TB, TC, R>), dim3((unsigned)blocks), dim3(256), 0, st, g);
    return hipGetLastError();
}

}  // namespace lmmse
