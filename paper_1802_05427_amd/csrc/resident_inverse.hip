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
    __asm__ volatile("" : "+s"(c));
    return c;
}

__device__ __forceinline__ double2 ri_shfl(double2 v, int src) {
    return make_double2(__shfl(v.x, src), __shfl(v.y, src));
}

// Sweep of the 16 pivots of one 16 x 16 sub-tile held in the result layout
// (re[v], im[v]: row 4 v + lk, column li), single pivots in order:
//   a_pp -> -1/d, a_pj -> a_pj / d, a_ip -> a_ip / d,
//   a_ij -> a_ij - a_ip a_pj / d        (d = a_pp),
// then its Hermitian part.  Returns false when a pivot is not positive and
// finite.  dt: the wave's 16 x kRiS LDS staging block, which ends holding the
// result row-major.
__device__ __forceinline__ bool ri_sweep_diag(zd4& re, zd4& im, double2 (*dt)[kRiS], int li, int lk) {
    bool ok = true;
    for (int p = 0; p < 16; ++p) {
        const int vp = p >> 2, lp = p & 3;   // wave-uniform
        // row p (as it is before this pivot), entry of this lane's column
        const double rx = vp == 0 ? re[0] : vp == 1 ? re[1] : vp == 2 ? re[2] : re[3];
        const double ry = vp == 0 ? im[0] : vp == 1 ? im[1] : vp == 2 ? im[2] : im[3];
        const double2 apj = ri_shfl(make_double2(rx, ry), 16 * lp + li);
        const double d = __shfl(rx, 16 * lp + p);
        ok = ok && d > 0.0 && isfinite(d);
        const double invd = 1.0 / d;
        const double2 q = make_double2(apj.x * invd, apj.y * invd);
        const bool jp = li == p;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            // a_ip of this lane's row 4 v + lk, read before element v changes
            const double2 aip = ri_shfl(make_double2(re[v], im[v]), 16 * lk + p);
            const bool ip = 4 * v + lk == p;
            // per-lane selects, not branches
            const double gx = fma(-aip.x, q.x, fma(aip.y, q.y, re[v]));
            const double gy = fma(-aip.x, q.y, fma(-aip.y, q.x, im[v]));
            re[v] = ip ? (jp ? -invd : q.x) : (jp ? aip.x * invd : gx);
            im[v] = ip ? (jp ? 0.0 : q.y) : (jp ? aip.y * invd : gy);
        }
    }
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

template <int NT>
__global__ __launch_bounds__(kRiThreads) void resident_inverse_kernel(double2* a, int n, double lam,
                                                                      int* status, long long mat0) {
    constexpr int NS = NT * (NT + 1) / 2;
    constexpr int SL = (NS + kRiWaves - 1) / kRiWaves;
    __shared__ double2 Pt[NT][16][kRiS];   // Pt[I][kk][r] = P_I[r][kk]
    __shared__ double2 Ft[NT][16][kRiS];   // Ft[I][kk][r] = F_I[r][kk]
    __shared__ double2 Dt[16][kRiS];       // D row-major
    __shared__ int bad;

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
    // Loads straight into the accumulators (real and imaginary parts as
    // separate 8-byte loads, so no staging registers), all issued before any
    // is used; then padding and lam on the diagonal.  Elements outside the
    // matrix read its element 0 and are replaced.
    zd4 cre[SL], cim[SL];
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
    __syncthreads();

#pragma unroll 1
    for (int k = 0; k < NT; ++k) {
        // 1. P of the panel's sub-tiles, and the sweep of the diagonal one
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
            }
        }
        {
            // the diagonal sub-tile, if this wave holds it (slot ud)
            int ud = -1;
#pragma unroll
            for (int u = 0; u < SL; ++u)
                if (code[u] == (k | k << 4 | 1 << 8)) ud = u;
            if (ud >= 0) {
                zd4 tr = cre[0], ti = cim[0];
#pragma unroll
                for (int u = 1; u < SL; ++u)
                    if (u == ud) {
                        tr = cre[u];
                        ti = cim[u];
                    }
                if (!ri_sweep_diag(tr, ti, Dt, li, lk) && lane == 0) bad = 1;
#pragma unroll
                for (int u = 0; u < SL; ++u)
                    if (u == ud) {
                        cre[u] = tr;
                        cim[u] = ti;
                    }
            }
        }
        __syncthreads();
        if (bad) {   // uniform: every wave leaves here
            if (tid == 0 && atomicCAS(status, 0, LMMSE_ERR_NOT_PD) == 0) status[1] = (int)(mat + mat0);
            return;
        }
        // 2. F of the panel's sub-tiles
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), cI = c & 15, cJ = (c >> 4) & 15;
            if (!(c >> 8)) continue;
            const bool col = cJ == k && cI > k, row = cI == k && cJ < k;
            if (!col && !row) continue;
            const int I = col ? cI : cJ;
            zd4 fr = {0, 0, 0, 0}, fi = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int kk = 4 * ks + lk;
                const double2 pv = Pt[I][kk][li];   // P_I[li][kk]
                if (col) {   // F_I = -P_I D: A = P_I[li][kk], B = D[kk][li]
                    const double2 dv = Dt[kk][li];
                    fr = __builtin_amdgcn_mfma_f64_16x16x4f64(-pv.x, dv.x, fr, 0, 0, 0);
                    fr = __builtin_amdgcn_mfma_f64_16x16x4f64(pv.y, dv.y, fr, 0, 0, 0);
                    fi = __builtin_amdgcn_mfma_f64_16x16x4f64(-pv.x, dv.y, fi, 0, 0, 0);
                    fi = __builtin_amdgcn_mfma_f64_16x16x4f64(-pv.y, dv.x, fi, 0, 0, 0);
                } else {     // F_J^H = -D P_J^H: A = D[li][kk], B = conj(P_J[li][kk])
                    const double2 dv = Dt[li][kk];
                    fr = __builtin_amdgcn_mfma_f64_16x16x4f64(-dv.x, pv.x, fr, 0, 0, 0);
                    fr = __builtin_amdgcn_mfma_f64_16x16x4f64(-dv.y, pv.y, fr, 0, 0, 0);
                    fi = __builtin_amdgcn_mfma_f64_16x16x4f64(dv.x, pv.y, fi, 0, 0, 0);
                    fi = __builtin_amdgcn_mfma_f64_16x16x4f64(-dv.y, pv.x, fi, 0, 0, 0);
                }
            }
            cre[u] = fr;
            cim[u] = fi;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (col)   // F_I[4v + lk][li]
                    Ft[I][li][4 * v + lk] = make_double2(fr[v], fi[v]);
                else       // F_J[li][4v + lk] = conj(F_J^H[4v + lk][li])
                    Ft[I][4 * v + lk][li] = make_double2(fr[v], -fi[v]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
        // 3. C -= F_I P_J^H off the panel's row and column
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const int c = ri_opaque(code[u]), I = c & 15, J = (c >> 4) & 15;
            if (!(c >> 8) || I == k || J == k) continue;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int kk = 4 * ks + lk;
                const double2 fv = Ft[I][kk][li];   // F_I[li][kk]
                const double2 pv = Pt[J][kk][li];   // P_J[li][kk]: B = conj
                cre[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fv.x, pv.x, cre[u], 0, 0, 0);
                cre[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fv.y, pv.y, cre[u], 0, 0, 0);
                cim[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fv.y, pv.x, cim[u], 0, 0, 0);
                cim[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(fv.x, pv.y, cim[u], 0, 0, 0);
            }
            // one slot's operands at a time: reading ahead for every slot
            // would hold 32 registers per slot
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();   // Pt, Ft and Dt are rewritten by the next panel
    }

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

// Sub-tile rows of the instantiated kernels (n <= 16 NT).
constexpr int kRiNT[] = {4, 6, 8, 10, 11, 12, 13};

bool resident_inverse_fits(int n) { return n >= 1 && n <= 16 * 13; }

hipError_t launch_resident_inverse(long long nmat, long long mat0, int n, double lam, double2* amat,
                                   int* status, hipStream_t st) {
    if (nmat == 0) return hipSuccess;
    if (!resident_inverse_fits(n)) return hipErrorInvalidValue;
    int nt = 0;
    for (int c : kRiNT)
        if (16 * c >= n) {
            nt = c;
            break;
        }
    const dim3 grid((unsigned)nmat), block(kRiThreads);
    switch (nt) {
#define LMMSE_RI(T) \
    case T: hipLaunchKernelGGL((resident_inverse_kernel<T>), grid, block, 0, st, amat, n, lam, status, mat0); break;
        LMMSE_RI(4) LMMSE_RI(6) LMMSE_RI(8) LMMSE_RI(10) LMMSE_RI(11) LMMSE_RI(12) LMMSE_RI(13)
#undef LMMSE_RI
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lmmse
