// -(A + lam I)^-1 of a Hermitian positive definite matrix held whole on one
// compute unit (n <= 16 NT, NT <= 13): the block solve of eq. 13 for windows
// up to 208 subcarriers (and the M x M systems of the push-through form) in
// one launch, without the window matrix going back to memory between panels.
//
// One workgroup of 8 waves per matrix.  The matrix (padded to 16 NT with the
// identity, whose inverse block is the identity again) is cut into 16 x 16
// sub-tiles; only the lower ones (I >= J) are kept, as FP64 matrix-core
// accumulators: sub-tile s = I (I + 1) / 2 + J lives in wave s % 8, slot
// s / 8, lane l holding rows 4 v + l / 16 (v < 4) of column l % 16 (the
// v_mfma_f64_16x16x4f64 result layout).  The upper sub-tiles are the
// conjugate transposes and are never formed.
//
// The Hermitian sweep then runs in panels of 16 pivots K = block k (rest R).
// Sweeping a panel at once maps
//     A_KK -> -A_KK^-1 = D,   A_RK -> F = A_RK A_KK^-1 = -P D,
//     A_RR -> A_RR - F P^H,   with P = A_RK before the step,
// which equals sweeping its pivots one by one.  Per panel:
//   1. the holders of the panel's sub-tiles publish P to LDS; the holder of
//      the diagonal sub-tile sweeps its 16 pivots in registers (rows and
//      columns of the pivot exchanged between lanes), replaces the result by
//      its Hermitian part (the rounding of the sweep is not Hermitian, and D
//      is used from both sides below) and publishes D;
//   2. every panel sub-tile becomes F_I = -P_I D (I > k) or F_J^H = -D P_J^H
//      (J < k, sub-tile (k, J)), on the matrix cores, and F goes to LDS;
//   3. every other sub-tile takes the rank-16 update C -= F_I P_J^H, four
//      real products per complex one, FP64 throughout.
// After the NT panels the sub-tiles hold -A^-1, which is written back in
// place (both triangles: each off-diagonal sub-tile and its mirror).
//
// The sample design of a window (COV): the kernel first forms A = X X^H / M
// + lam I itself from the LS values (FP32 matrix-core products, as the
// batched covariance product does them), and at the end writes the window's
// block filter rows W = I + lam S (S = -A^-1) straight from the registers,
// and A^-1 only when the backward needs it; the window matrix never goes to
// memory otherwise.
//
// Time: the rank-16 updates are bound by the FP64 matrix cores (one
// 16 x 16 x 4 product per SIMD every 64 cycles, whichever wave issues it);
// the one-wave sweep of each diagonal block and the barriers around it are
// the serial part.
#include "split.h"
#include "zgemm.h"

namespace lmmse {

constexpr int kRiWaves = 8;
constexpr int kRiThreads = 64 * kRiWaves;
constexpr int kRiS = 17;   // LDS row stride (complex values) of a staged 16 x 16 block

__device__ __forceinline__ void ri_wave_sync() {
    // orders one wave's LDS accesses across its lanes (no workgroup barrier)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A slot code made opaque to the compiler inside the panel loop, so that the
// addresses derived from it are formed where they are used rather than held
// in registers across the loop for every slot.
__device__ __forceinline__ int ri_opaque(int c) {
    c = __builtin_amdgcn_readfirstlane(c);   // uniform; a scalar register for the constraint
    __asm__ volatile("" : "+s"(c));
    return c;
}

__device__ __forceinline__ double2 ri_shfl(double2 v, int src) {
    return make_double2(__shfl(v.x, src), __shfl(v.y, src));
}

// Lane (li, lk) takes x of lane (P, lk): the DPP broadcast of one lane of
// every 16-lane row to its row (a register move, no LDS round trip).
template <int P>
__device__ __forceinline__ double ri_rowbcast(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x150 + P, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + P, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double ri_readlane(double x, int l) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// 1/d for a positive finite d: the hardware estimate refined by two Newton
// steps (each squares the relative error), well within an ulp or two of the
// quotient, with a short dependency chain.
__device__ __forceinline__ double ri_rcp(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    return fma(fma(-d, r, 1.0), r, r);
}

// Pivot P of the sweep of one 16 x 16 sub-tile held in the result layout
// (re[v], im[v]: row 4 v + lk, column li):
//   a_pp -> -1/d, a_pj -> a_pj / d, a_ip -> a_ip / d,
//   a_ij -> a_ij - a_ip a_pj / d        (d = a_pp).
// Column P reaches every lane of a row by DPP, row P (held by row-group
// P % 4, entry P / 4) by a lane permute, d by reading one lane.
template <int P>
__device__ __forceinline__ bool ri_pivot(zd4& re, zd4& im, int li, int lk) {
    constexpr int vp = P >> 2, lp = P & 3;
    const double d = ri_readlane(re[vp], 16 * lp + P);
    const double2 apj = ri_shfl(make_double2(re[vp], im[vp]), 16 * lp + li);
    double2 aip[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) aip[v] = make_double2(ri_rowbcast<P>(re[v]), ri_rowbcast<P>(im[v]));
    const double invd = ri_rcp(d);
    const double2 q = make_double2(apj.x * invd, apj.y * invd);
    const bool jp = li == P;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const bool ip = 4 * v + lk == P;
        // per-lane selects, not branches
        const double gx = fma(-aip[v].x, q.x, fma(aip[v].y, q.y, re[v]));
        const double gy = fma(-aip[v].x, q.y, fma(-aip[v].y, q.x, im[v]));
        re[v] = ip ? (jp ? -invd : q.x) : (jp ? aip[v].x * invd : gx);
        im[v] = ip ? (jp ? 0.0 : q.y) : (jp ? aip[v].y * invd : gy);
    }
    return d > 0.0 && isfinite(d);
}

template <int P>
__device__ __forceinline__ bool ri_pivots(zd4& re, zd4& im, int li, int lk) {
    const bool ok = ri_pivot<P>(re, im, li, lk);
    if constexpr (P + 1 < 16)
        return ri_pivots<P + 1>(re, im, li, lk) && ok;
    else
        return ok;
}

// Sweep of the 16 pivots of one 16 x 16 sub-tile in order, then its
// Hermitian part.  Returns false when a pivot is not positive and finite.
// dt: the wave's 16 x kRiS LDS staging block, which ends holding the result
// row-major.
__device__ __forceinline__ bool ri_sweep_diag(zd4& re, zd4& im, double2 (*dt)[kRiS], int li, int lk) {
    const bool ok = ri_pivots<0>(re, im, li, lk);
    // Hermitian part: entry (i, j) and conj of (j, i) through LDS
#pragma unroll
    for (int v = 0; v < 4; ++v) dt[4 * v + lk][li] = make_double2(re[v], im[v]);
    ri_wave_sync();
    double2 tr[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) tr[v] = dt[li][4 * v + lk];
    ri_wave_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        re[v] = 0.5 * (re[v] + tr[v].x);
        im[v] = 0.5 * (im[v] - tr[v].y);
        dt[4 * v + lk][li] = make_double2(re[v], im[v]);
    }
    return ok;
}

// The holder of a diagonal sub-tile (one wave), once the block is staged in
// dt: the block swept (the result, D = -block^-1, ends in dt; the slot takes
// it from there later).  A pivot that is not positive and finite sets bad.
__device__ __forceinline__ void ri_sweep_staged(double2 (*dt)[kRiS], int li, int lk, int& bad, int lane) {
    ri_wave_sync();
    zd4 tr, ti;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double2 x = dt[4 * v + lk][li];
        tr[v] = x.x;
        ti[v] = x.y;
    }
    ri_wave_sync();
    if (!ri_sweep_diag(tr, ti, dt, li, lk) && lane == 0) bad = 1;
}

// D = (+-A) (+-B) + C on the FP64 matrix cores; NEG bit 0 negates A, bit 1
// negates B (the instruction's own modifiers, so no separate negation).
template <int NEG>
__device__ __forceinline__ zd4 ri_mma(double a, double b, zd4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, NEG);
}

// C -= F P^H for one 16 x 16 sub-tile: A = F[li][kk] = ft[kk][li],
// B = (P^H)[kk][li] = conj(pt[kk][li]), four real products per complex one.
// f0, q0: the first step's operands, read ahead by the caller.
__device__ __forceinline__ void ri_update(zd4& cr, zd4& ci, const double2 (*ft)[kRiS],
                                          const double2 (*pt)[kRiS], double2 f0, double2 q0, int li,
                                          int lk) {
    double2 f = f0, q = q0;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        double2 fn = f, qn = q;
        if (ks + 1 < 4) {
            fn = ft[4 * (ks + 1) + lk][li];
            qn = pt[4 * (ks + 1) + lk][li];
        }
        cr = ri_mma<1>(f.x, q.x, cr);   // re -= fx qx + fy qy
        ci = ri_mma<1>(f.y, q.x, ci);   // im -= fy qx - fx qy
        cr = ri_mma<1>(f.y, q.y, cr);
        ci = ri_mma<0>(f.x, q.y, ci);
        f = fn;
        q = qn;
    }
}

// The window's LS values for the fused covariance: X[j][m] = h_ls[s, m, k,
// starts[b] + j] (complex FP32, [S][M][K][N]) for matrix (s K + k) nb + b.
struct RiCov {
    const float2* hls;
    const int* starts;
    int M, K, N, nb;
    // the block filters straight from the registers: W = (I + lam S)[off
    // rows] (S = -A^-1, off = offsets[b], B rows) into w64 [mat][B][Wn],
    // w32 [mat][B][Wn rounded up to 2] or whi / wlo [mat][B][Wn rounded up
    // to 4] (split, FP16 when fp16), any of them null; with ainv, A^-1 = -S
    // into the window matrix, which is otherwise not written
    const int* offsets;
    int B;
    double2* w64;
    float2* w32;
    uint32_t* whi;
    uint32_t* wlo;
    int fp16, ainv;
};

// Entry (o, col) of this window's block filter, w = delta + lam s.
__device__ __forceinline__ void ri_store_w(const RiCov& cv, long long mat, int o, int col, int n, double2 w) {
    const long long row = mat * cv.B + o;
    if (cv.w64) cv.w64[row * n + col] = w;
    if (cv.w32)   // FP32 filters: the chunk-major order of the split parts
        cv.w32[split_w_index(mat * cv.B * (long long)((n + 15) & ~15), cv.B, o, col)] =
            make_float2((float)w.x, (float)w.y);
    if (cv.whi) {
        uint32_t h, l;
        const float2 wf = make_float2((float)w.x, (float)w.y);
        if (cv.fp16)
            split_c<true>(wf, h, l);
        else
            split_c<false>(wf, h, l);
        const long long i = split_w_index(mat * cv.B * (long long)((n + 15) & ~15), cv.B, o, col);
        cv.whi[i] = h;
        cv.wlo[i] = l;
    }
}

typedef float ri_f4 __attribute__((ext_vector_type(4)));

// R = X X^H / M on the FP32 matrix cores for this wave's lower sub-tiles,
// then A = R + lam I (identity on the padding) in the FP64 layout of the
// inverse: the same products, in the same order, with FP32 sums over the
// antennas, as the batched covariance product of the wider windows.  The LS
// values go through LDS in chunks of 16 antennas (xs: two [16][16 NT]
// buffers), the next chunk read into registers during the current one's
// products.  The FP32 result layout (row 4 lk + v) is turned into the FP64
// one (row 4 v + lk) through the wave's own LDS block tw.
template <int NT, int SL>
__device__ __forceinline__ void ri_covariance(zd4 (&cre)[SL], zd4 (&cim)[SL], const int (&code)[SL],
                                              const RiCov& cv, long long mat, int n, double lam,
                                              float2* xs, double2 (*tw)[kRiS], int tid, int lane) {
    constexpr int R = 16 * NT;                        // rows of a chunk
    constexpr int PT = (16 * R + kRiThreads - 1) / kRiThreads;   // chunk values per thread
    const int li = lane & 15, lk = lane >> 4;
    const int b = (int)(mat % cv.nb);
    const long long sk = mat / cv.nb;
    const float2* xw = cv.hls + (sk / cv.K) * ((long long)cv.M * cv.K * cv.N) + (sk % cv.K) * cv.N +
                       cv.starts[b];
    const long long ms = (long long)cv.K * cv.N;   // antenna stride
    float2 pre[PT];
    auto fetch = [&](int m0) {
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int e = tid + kRiThreads * t, m = e / R, j = e - m * R;
            const bool ok = e < 16 * R && j < n && m0 + m < cv.M;
            pre[t] = xw[ok ? (m0 + m) * ms + j : 0];
            if (!ok) pre[t] = make_float2(0.f, 0.f);
        }
    };
    ri_f4 fr[SL], fi[SL];
#pragma unroll
    for (int u = 0; u < SL; ++u) {
        fr[u] = ri_f4{0, 0, 0, 0};
        fi[u] = ri_f4{0, 0, 0, 0};
    }
    fetch(0);
    const int nch = (cv.M + 15) / 16;
    for (int ch = 0; ch < nch; ++ch) {
        float2* xb = xs + (ch & 1) * 16 * R;   // [16 antennas][R rows]
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int e = tid + kRiThreads * t;
            if (e < 16 * R) xb[e] = pre[t];
        }
        __syncthreads();   // (the other buffer was last read before the previous barrier)
        if (ch + 1 < nch) fetch(16 * (ch + 1));
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
            if (!(c >> 8)) continue;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const float2 x1 = xb[(4 * ks + lk) * R + 16 * I + li], x2 = xb[(4 * ks + lk) * R + 16 * J + li];
                // x1 conj(x2): re = x1.x x2.x + x1.y x2.y, im = x1.y x2.x - x1.x x2.y
                fr[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.x, x2.x, fr[u], 0, 0, 0);
                fr[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.y, x2.y, fr[u], 0, 0, 0);
                fi[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(-x1.x, x2.y, fi[u], 0, 0, 0);
                fi[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.y, x2.x, fi[u], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const double invM = 1.0 / cv.M;
#pragma unroll
    for (int u = 0; u < SL; ++u) {
        const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
#pragma unroll
        for (int v = 0; v < 4; ++v) tw[4 * lk + v][li] = make_double2(invM * fr[u][v], invM * fi[u][v]);
        ri_wave_sync();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double2 x = tw[4 * v + lk][li];
            const int i = 16 * I + 4 * v + lk, j = 16 * J + li;
            const bool ok = (c >> 8) && i < n && j < n;
            const double dg = i == j ? (ok ? lam : 1.0) : 0.0;   // padding: identity
            cre[u][v] = (ok ? x.x : 0.0) + dg;
            cim[u][v] = ok ? x.y : 0.0;
        }
        ri_wave_sync();
    }
}

// The same with FP64 products and sums on the FP64 matrix cores (the
// products of FP32 values are exact in FP64): for windows up to 160, whose
// covariance keeps FP64 sums.  The accumulators are the slots themselves,
// already in the inverse's layout.
template <int NT, int SL>
__device__ __forceinline__ void ri_covariance64(zd4 (&cre)[SL], zd4 (&cim)[SL], const int (&code)[SL],
                                                const RiCov& cv, long long mat, int n, double lam,
                                                float2* xs, int tid, int lane) {
    constexpr int R = 16 * NT;
    constexpr int PT = (16 * R + kRiThreads - 1) / kRiThreads;
    const int li = lane & 15, lk = lane >> 4;
    const int b = (int)(mat % cv.nb);
    const long long sk = mat / cv.nb;
    const float2* xw = cv.hls + (sk / cv.K) * ((long long)cv.M * cv.K * cv.N) + (sk % cv.K) * cv.N +
                       cv.starts[b];
    const long long ms = (long long)cv.K * cv.N;
    float2 pre[PT];
    auto fetch = [&](int m0) {
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int e = tid + kRiThreads * t, m = e / R, j = e - m * R;
            const bool ok = e < 16 * R && j < n && m0 + m < cv.M;
            pre[t] = xw[ok ? (m0 + m) * ms + j : 0];
            if (!ok) pre[t] = make_float2(0.f, 0.f);
        }
    };
#pragma unroll
    for (int u = 0; u < SL; ++u) {
        cre[u] = zd4{0, 0, 0, 0};
        cim[u] = zd4{0, 0, 0, 0};
    }
    fetch(0);
    const int nch = (cv.M + 15) / 16;
    for (int ch = 0; ch < nch; ++ch) {
        float2* xb = xs + (ch & 1) * 16 * R;
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int e = tid + kRiThreads * t;
            if (e < 16 * R) xb[e] = pre[t];
        }
        __syncthreads();
        if (ch + 1 < nch) fetch(16 * (ch + 1));
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
            if (!(c >> 8)) continue;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const float2 x1 = xb[(4 * ks + lk) * R + 16 * I + li], x2 = xb[(4 * ks + lk) * R + 16 * J + li];
                const double ax = x1.x, ay = x1.y, bx = x2.x, by = x2.y;
                // x1 conj(x2): re = ax bx + ay by, im = ay bx - ax by
                cre[u] = ri_mma<0>(ax, bx, cre[u]);
                cim[u] = ri_mma<0>(ay, bx, cim[u]);
                cre[u] = ri_mma<0>(ay, by, cre[u]);
                cim[u] = ri_mma<1>(ax, by, cim[u]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const double invM = 1.0 / cv.M;
#pragma unroll
    for (int u = 0; u < SL; ++u) {
        const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + 4 * v + lk, j = 16 * J + li;
            const bool ok = (c >> 8) && i < n && j < n;
            const double dg = i == j ? (ok ? lam : 1.0) : 0.0;   // padding: identity
            cre[u][v] = (ok ? invM * cre[u][v] : 0.0) + dg;
            cim[u][v] = ok ? invM * cim[u][v] : 0.0;
        }
    }
}

template <int NT, int COV>
__global__ __launch_bounds__(kRiThreads) void resident_inverse_kernel(double2* a, int n, double lam,
                                                                      int* status, long long mat0,
                                                                      RiCov cv) {
    constexpr int NS = NT * (NT + 1) / 2;
    constexpr int SL = (NS + kRiWaves - 1) / kRiWaves;
    constexpr int kBlk = 16 * kRiS;   // one staged 16 x 16 block (complex values)
    // Pt[I][kk][r] = P_I[r][kk], Ft[I][kk][r] = F_I[r][kk], Dt = D row-major;
    // while the covariance is formed, Pt's area holds the LDS chunks of the
    // LS values and Ft's the per-wave blocks of the layout change
    __shared__ double2 lds_all[(2 * NT + 1) * kBlk];
    __shared__ int bad;
    double2(*Pt)[16][kRiS] = reinterpret_cast<double2(*)[16][kRiS]>(lds_all);
    double2(*Ft)[16][kRiS] = reinterpret_cast<double2(*)[16][kRiS]>(lds_all + NT * kBlk);
    double2(*Dt)[kRiS] = reinterpret_cast<double2(*)[kRiS]>(lds_all + 2 * NT * kBlk);

    const long long mat = blockIdx.x;
    double2* am = a + mat * n * n;
    const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    if (tid == 0) bad = 0;

    // slot u of this wave: sub-tile s = w + 8 u -> (I, J), packed as
    // I | J << 4 | live << 8 (unused slots, s >= NS, read element 0 and are
    // never updated or written)
    int code[SL];
#pragma unroll
    for (int u = 0; u < SL; ++u) {
        int s = w + kRiWaves * u, I = 0;
        const int lv = s < NS ? 1 : 0;
        if (!lv) s = 0;
        while (s > I) {
            s -= I + 1;
            ++I;
        }
        code[u] = I | s << 4 | lv << 8;
    }
    zd4 cre[SL], cim[SL];
    if constexpr (COV == 1) {
        ri_covariance<NT, SL>(cre, cim, code, cv, mat, n, lam, reinterpret_cast<float2*>(lds_all),
                              reinterpret_cast<double2(*)[16][kRiS]>(lds_all + NT * kBlk)[w], tid, lane);
    } else if constexpr (COV == 2) {
        ri_covariance64<NT, SL>(cre, cim, code, cv, mat, n, lam, reinterpret_cast<float2*>(lds_all), tid, lane);
    } else {
        // Loads straight into the accumulators (real and imaginary parts as
        // separate 8-byte loads, so no staging registers), all issued before
        // any is used; then padding and lam on the diagonal.  Elements outside
        // the matrix read its element 0 and are replaced.
        const double* ad = reinterpret_cast<const double*>(am);
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + 4 * v + lk, j = 16 * J + li;
                const long long e = (c >> 8) && i < n && j < n ? (long long)i * n + j : 0;
                cre[u][v] = ad[2 * e];
                cim[u][v] = ad[2 * e + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + 4 * v + lk, j = 16 * J + li;
                const bool ok = (c >> 8) && i < n && j < n;
                const double dg = i == j ? (ok ? lam : 1.0) : 0.0;   // padding: identity
                cre[u][v] = (ok ? cre[u][v] : 0.0) + dg;
                cim[u][v] = ok ? cim[u][v] : 0.0;
            }
        }
    }
    __syncthreads();

#pragma unroll 1
    for (int k = 0; k < NT; ++k) {
        // 1. P of the panel's sub-tiles and the diagonal block to LDS; the
        //    holder of the diagonal block sweeps it there (D = -A_KK^-1)
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
            if (!(c >> 8)) continue;
            if (I == k && J < k) {   // (k, J): P_J[r][kk] = conj(C[kk][r])
#pragma unroll
                for (int v = 0; v < 4; ++v) Pt[J][4 * v + lk][li] = make_double2(cre[u][v], -cim[u][v]);
            } else if (J == k && I > k) {   // (I, k): P_I[r][kk] = C[r][kk]
#pragma unroll
                for (int v = 0; v < 4; ++v) Pt[I][li][4 * v + lk] = make_double2(cre[u][v], cim[u][v]);
            } else if (I == k && J == k) {
#pragma unroll
                for (int v = 0; v < 4; ++v) Dt[4 * v + lk][li] = make_double2(cre[u][v], cim[u][v]);
            }
        }
        if (w == (k * (k + 3) / 2) % kRiWaves) ri_sweep_staged(Dt, li, lk, bad, lane);
        __syncthreads();
        if (bad) {   // uniform: every wave leaves here
            if (tid == 0 && atomicCAS(status, 0, LMMSE_ERR_NOT_PD) == 0) status[1] = (int)(mat + mat0);
            return;
        }
        // 2. the panel's sub-tiles: F_I = -P_I D for (I, k), I > k, and
        //    F_J^H = -D P_J^H for (k, J), J < k (the choice made once per slot:
        //    a branch inside the product made the compiler copy the
        //    accumulators around it); then D itself into sub-tile (k, k)
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), cI = c & 15, cJ = (c >> 4) & 15;
            if (!(c >> 8)) continue;
            const bool col = cJ == k && cI > k, row = cI == k && cJ < k;
            if (!col && !row) continue;
            cre[u] = zd4{0, 0, 0, 0};
            cim[u] = zd4{0, 0, 0, 0};
            if (col) {   // F_I = -P_I D: A = P_I[li][kk], B = D[kk][li]
                const int I = cI;
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int kk = 4 * ks + lk;
                    const double2 av = Pt[I][kk][li], bv = Dt[kk][li];
                    cre[u] = ri_mma<1>(av.x, bv.x, cre[u]);
                    cim[u] = ri_mma<1>(av.x, bv.y, cim[u]);
                    cre[u] = ri_mma<0>(av.y, bv.y, cre[u]);
                    cim[u] = ri_mma<1>(av.y, bv.x, cim[u]);
                }
#pragma unroll   // F_I[4v + lk][li] -> Ft[I][li][4v + lk]
                for (int v = 0; v < 4; ++v) Ft[I][li][4 * v + lk] = make_double2(cre[u][v], cim[u][v]);
            } else {     // F_J^H = -D P_J^H: A = D[li][kk], B = conj(P_J[li][kk])
                const int J = cJ;
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int kk = 4 * ks + lk;
                    const double2 av = Dt[li][kk], bv = Pt[J][kk][li];
                    cre[u] = ri_mma<1>(av.x, bv.x, cre[u]);
                    cim[u] = ri_mma<0>(av.x, bv.y, cim[u]);
                    cre[u] = ri_mma<1>(av.y, bv.y, cre[u]);
                    cim[u] = ri_mma<1>(av.y, bv.x, cim[u]);
                }
#pragma unroll   // F_J[li][4v + lk] = conj(F_J^H[4v + lk][li]) -> Ft[J][4v + lk][li]
                for (int v = 0; v < 4; ++v) Ft[J][4 * v + lk][li] = make_double2(cre[u][v], -cim[u][v]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            if (ri_opaque(code[u]) != (k | k << 4 | 1 << 8)) continue;
            __asm__ volatile("");   // a branch, not selects over every slot
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double2 x = Dt[4 * v + lk][li];
                cre[u][v] = x.x;
                cim[u][v] = x.y;
            }
        }
        __syncthreads();
        // 3. C -= F_I P_J^H off the panel's row and column.  The first step's
        //    operands of the next slot are read during this slot's products
        //    (every slot's indices are valid, active or not), so that a wave,
        //    which issues an FP64 product only every other turn of its SIMD,
        //    does not wait on LDS between slots.
        double2 f0 = Ft[code[0] & 15][lk][li], q0 = Pt[(code[0] >> 4) & 15][lk][li];
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
            double2 fn = f0, qn = q0;
            if (u + 1 < SL) {
                const int cn = ri_opaque(code[u + 1]);
                fn = Ft[cn & 15][lk][li];
                qn = Pt[(cn >> 4) & 15][lk][li];
            }
            if ((c >> 8) && I != k && J != k) ri_update(cre[u], cim[u], Ft[I], Pt[J], f0, q0, li, lk);
            f0 = fn;
            q0 = qn;
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();   // Pt, Ft and Dt are rewritten by the next panel
    }

    if constexpr (COV != 0) {
        // the block filter rows (each sub-tile's kept rows, and those of the
        // mirror of an off-diagonal one), their padding columns, and A^-1
        // when asked for
        const int off = cv.offsets[mat % cv.nb];
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
            if (!(c >> 8)) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + 4 * v + lk, j = 16 * J + li;
                if (i >= n || j >= n) continue;
                const double sx = cre[u][v], sy = cim[u][v];
                if (cv.ainv) {
                    am[(long long)i * n + j] = make_double2(-sx, -sy);
                    if (I != J) am[(long long)j * n + i] = make_double2(-sx, sy);
                }
                if (i >= off && i < off + cv.B)
                    ri_store_w(cv, mat, i - off, j, n, make_double2((i == j ? 1.0 : 0.0) + lam * sx, lam * sy));
                if (I != J && j >= off && j < off + cv.B)
                    ri_store_w(cv, mat, j - off, i, n, make_double2(lam * sx, -lam * sy));
            }
        }
        const int pad = (cv.whi || cv.w32) ? ((n + 15) & ~15) - n : 0;
        for (int e = tid; e < cv.B * pad; e += kRiThreads) {
            const int o = e / pad, col = n + e % pad;
            const long long i = split_w_index(mat * cv.B * (long long)(n + pad), cv.B, o, col);
            if (cv.whi) {
                cv.whi[i] = 0u;
                cv.wlo[i] = 0u;
            } else {
                cv.w32[i] = make_float2(0.f, 0.f);
            }
        }
    } else {
        // -A^-1 back in place: each sub-tile, and the mirror of an off-diagonal one
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
            if (!(c >> 8)) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + 4 * v + lk, j = 16 * J + li;
                if (i < n && j < n) {
                    am[(long long)i * n + j] = make_double2(cre[u][v], cim[u][v]);
                    if (I != J) am[(long long)j * n + i] = make_double2(cre[u][v], -cim[u][v]);
                }
            }
        }
    }
}

// Sub-tile rows of the instantiated kernels (n <= 16 NT).
constexpr int kRiNT[] = {4, 8, 10, 11, 12, 13};

bool resident_inverse_fits(int n) { return n >= 1 && n <= 16 * 13; }

// cov: when not null, A = X X^H / M + lam I is formed from the LS values in
// the kernel and the block filters written from it (the window matrices in
// amat are then output only): FP64 products and sums (cov64, windows of
// 129..160) or FP32 ones (161..208).
static hipError_t launch_ri(long long nmat, long long mat0, int n, double lam, double2* amat, int* status,
                            const RiCov* cov, bool cov64, hipStream_t st) {
    if (nmat == 0) return hipSuccess;
    if (!resident_inverse_fits(n)) return hipErrorInvalidValue;
    // one workgroup per matrix in a single grid, whose work-items must stay
    // below 2^32 (about 8.4 million matrices)
    if (nmat > (long long)(0xFFFFFFFFu / kRiThreads)) return hipErrorInvalidValue;
    int nt = 0;
    for (int c : kRiNT)
        if (16 * c >= n) {
            nt = c;
            break;
        }
    const dim3 grid((unsigned)nmat), block(kRiThreads);
    const RiCov cv = cov ? *cov : RiCov{};
    if (cov && cov64) {
        if (nt != 10) return hipErrorInvalidValue;
        hipLaunchKernelGGL((resident_inverse_kernel<10, 2>), grid, block, 0, st, amat, n, lam, status, mat0, cv);
    } else if (cov) {
        switch (nt) {
#define LMMSE_RIC(T) \
    case T: hipLaunchKernelGGL((resident_inverse_kernel<T, 1>), grid, block, 0, st, amat, n, lam, status, mat0, cv); break;
            LMMSE_RIC(11) LMMSE_RIC(12) LMMSE_RIC(13)
#undef LMMSE_RIC
            default:
                return hipErrorInvalidValue;
        }
    } else {
        switch (nt) {
#define LMMSE_RI(T) \
    case T: hipLaunchKernelGGL((resident_inverse_kernel<T, 0>), grid, block, 0, st, amat, n, lam, status, mat0, cv); break;
            LMMSE_RI(4) LMMSE_RI(8) LMMSE_RI(10) LMMSE_RI(11) LMMSE_RI(12) LMMSE_RI(13)
#undef LMMSE_RI
            default:
                return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_resident_inverse(long long nmat, long long mat0, int n, double lam, double2* amat,
                                   int* status, hipStream_t st) {
    return launch_ri(nmat, mat0, n, lam, amat, status, nullptr, false, st);
}

bool resident_design_fits(int Wn) { return Wn > kResidentFp64Cov && resident_inverse_fits(Wn); }

hipError_t launch_resident_design(const Plan& p, long long nmat, long long mat0, const float2* hls, double lam,
                                  double2* amat, double2* w64, float2* w32, uint32_t* whi, uint32_t* wlo,
                                  bool want_ainv, hipStream_t st) {
    if (!resident_design_fits(p.d.Wn)) return hipErrorInvalidValue;
    if ((whi == nullptr) != (wlo == nullptr) || (whi && w32)) return hipErrorInvalidValue;
    const RiCov cv{hls, p.d_starts, p.d.M, p.d.K, p.d.N, p.nb, p.d_offsets, p.d.B, w64, w32, whi, wlo,
                   p.d.precision == LMMSE_FP16X3 ? 1 : 0, want_ainv ? 1 : 0};
    // windows up to 160 keep FP64 sums in their covariance
    return launch_ri(nmat, mat0, p.d.Wn, lam, amat, p.status, &cv, p.d.Wn <= kMaxSampleWindowReg, st);
}

}  // namespace lmmse
