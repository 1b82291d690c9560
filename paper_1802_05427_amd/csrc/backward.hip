// Backward pass of the fixed-design estimator (gradients through eq. 12 and
// the eq. 13 / eq. 17 block filters of Sec. IV-B).
//
// Convention: g = dL/dRe(Hhat) + j dL/dIm(Hhat).  For block b with filter W
// (B x Wn), window X_b (Wn values per column) and outputs G_b:
//   d X_b  += W^H G_b                          (dx kernels)
//   dW_c    = sum over blocks b of class c and all columns of G_b X_b^H
//   Z_c     = dW_c A^-1,   Gamma_II = -W_c^H Z_c,   Gamma_OI = Z_c
//   dlam    = sum_c Re tr(Gamma_II)
//   dtau    = sum_c Re [ sum conj(Z_c) dR_OI + sum conj(Gamma_II) dR_II ]
// with A = R_II + lam I, R entries r_{i-j} and dR = d r / d tau.
//
// dX: the FP32 filtering kernel of the forward pass with transposed roles
// (apply_f32.hip): contraction over the B outputs of each block, Wn output
// rows, the real embedding of W^H as its bank.  Windows of neighbouring
// blocks overlap, so the blocks are processed in passes whose windows are
// disjoint (block b in pass b mod P): the first pass stores its windows, the
// subcarriers none of them covers are zeroed, and each later pass adds its
// contribution with a read-add-write: deterministic, no atomics.
//
// dW: split over column chunks.  A workgroup takes one block, one row group of
// its 2B real output rows and one chunk of columns; wave w owns window columns
// [16w, 16w+16) of dW_b and all row tiles of the group.  16 LS columns at a
// time, G_b and X_b are staged in LDS transposed (column index fastest), so
// that each MFMA operand is one 16-byte read: A is the real embedding of G
// built in registers, B is X interleaved, contracted over (column, re/im).
// The next 16 columns are loaded into registers before the MFMAs of the
// current ones.  Each workgroup writes its FP32 partial; the partials are
// summed per class in FP64 in a fixed order.
#include <algorithm>

#include "internal.h"

namespace lmmse {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bq(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// ---------------------------------------------------------------- layout sizes
struct BwGeom {
    int RT, rgroups, Rpad;   // dX: row tiles over the 2Wn real rows of W^H
    int G16b;                // dX: chunks of 16 block outputs (contraction)
    int P;                   // passes with disjoint windows
    int dwRT, dwRG;          // dW: row tiles per workgroup, row groups
    int nch;                 // column chunks of the dW reduction
    long long cpw;           // columns per chunk (multiple of 16)
};

constexpr int kDwMaxRT = 13;          // dW row tiles per workgroup (2B real rows in row groups):
                                      // one group for B <= 104, so the window is read once;
                                      // <= 128 registers, 4 waves per SIMD
constexpr int kDwMaxWaves = 16;       // one wave per 16 window columns: Wn <= 256
static_assert(16 * kDwMaxWaves == kMaxSampleWindowLarge,
              "lmmse_backward refuses design gradients above kMaxSampleWindowLarge");
constexpr int kDwSlots = 256;         // workgroups resident at once (one 10-wave workgroup per CU at Wn = 150)

static BwGeom bw_geom(const lmmse_plan_desc& d, const std::vector<int>& starts, long long ncols) {
    BwGeom g{};
    transposed_row_tiles(d.Wn, g.RT, g.rgroups);
    g.Rpad = g.RT * 16 * g.rgroups;
    g.G16b = (d.B + 15) / 16;
    const int nb = (int)starts.size();
    g.P = 1;
    for (bool clash = true; clash;) {
        clash = false;
        for (int b = 0; b + g.P < nb; ++b)
            if (starts[b + g.P] < starts[b] + d.Wn) clash = true;
        if (clash) ++g.P;
    }
    const int tw = (2 * d.B + 15) / 16;
    g.dwRG = (tw + kDwMaxRT - 1) / kDwMaxRT;
    g.dwRT = (tw + g.dwRG - 1) / g.dwRG;
    // one resident wave of workgroups; at least 16 columns per chunk
    const long long steps = (ncols + 15) / 16;
    if (steps == 0) {   // empty batch: no chunks
        g.nch = 0;
        g.cpw = 16;
        return g;
    }
    const long long want = std::max(1, kDwSlots / (nb * g.dwRG));
    g.nch = (int)std::max(1LL, std::min(want, steps));
    g.cpw = 16 * ((steps + g.nch - 1) / g.nch);
    g.nch = (int)((ncols + g.cpw - 1) / g.cpw);
    return g;
}

// ---------------------------------------------------------------- W^H bank
// Real embedding of W^H (2Wn x 2B): Wr'[2i+ri][2o+ro] from conj(W[o][i]), in
// the FP32 bank order of the filtering kernel: groups g < 2 ceil(B/16) of 8
// block outputs, row groups of RT*16 rows, lanes q:
// bank[(((c*ngroups + g)*rgroups + rg)*4 + q)*RT*16 + rr] = Wr'[rg*RT*16 + rr][16g + 4q .. +3].
__global__ void pack_wh_kernel(const double2* __restrict__ w64, float4* __restrict__ bank,
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
    const int i = r >> 1, ri = r & 1;
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int kr = 16 * g + 4 * q + e;
        const int o = kr >> 1, ro = kr & 1;
        float x = 0.f;
        if (i < Wn && o < B) {
            const double2 w = w64[((long long)c * B + o) * Wn + i];   // W^H[i][o] = conj(w)
            if (ri == 0) x = (float)(ro == 0 ? w.x : w.y);
            else x = (float)(ro == 0 ? -w.y : w.x);
        }
        v[e] = x;
    }
    bank[idx] = make_float4(v[0], v[1], v[2], v[3]);
}

__global__ void fill_zero_kernel(float2* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_float2(0.f, 0.f);
}

// Subcarrier runs [lo, lo + len) that no window of the first dX pass covers;
// off[i] = total length of runs before run i.
constexpr int kMaxGapRuns = 64;
struct GapRuns {
    int lo[kMaxGapRuns], off[kMaxGapRuns + 1];
    int n;
};

// dX = 0 on the runs of every column (one thread per zeroed element).
__global__ void fill_gaps_kernel(float2* dx, long long ncols, int N, GapRuns gr) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int tot = gr.off[gr.n];
    if (e >= ncols * tot) return;
    const long long col = e / tot;
    const int k = (int)(e - col * tot);
    int i = 0;
    while (i + 1 < gr.n && gr.off[i + 1] <= k) ++i;
    dx[col * N + gr.lo[i] + (k - gr.off[i])] = make_float2(0.f, 0.f);
}

// ---------------------------------------------------------------- dW partials
struct DwArgs {
    const int* starts;
    const float2* g;
    const float2* x;
    float2* part;        // [nb][nch][B][Wn]
    long long ncols, cpw;
    int N, B, Wn, nb, nch, rgroups;
};

constexpr int kDwS = 18;   // LDS row stride (float2) of the transposed tiles: 16 columns + pad

template <int RT>
__global__ __launch_bounds__(64 * kDwMaxWaves) __attribute__((amdgpu_waves_per_eu(4)))
void dw_kernel(DwArgs a) {
    constexpr int NO = RT * 8;                     // complex output rows of the group
    __shared__ float2 gT[NO * kDwS];               // G: [o][col]
    __shared__ float2 xT[16 * kDwMaxWaves * kDwS]; // X: [j][col]
    const int nthr = blockDim.x;
    const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, q = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    long long t = blockIdx.x;
    const int rg = (int)(t % a.rgroups);
    t /= a.rgroups;
    const int b = (int)(t % a.nb);
    const int ch = (int)(t / a.nb);
    const int s0 = a.starts[b];
    const int o0 = rg * NO;                        // first output row of the group
    const long long col_lo = (long long)ch * a.cpw;
    const long long col_hi = min(col_lo + a.cpw, a.ncols);
    const int nsteps = (int)((col_hi - col_lo + 15) / 16);
    // Staging: the 16 x NO tile of G and the 16 x Wn tile of X are cut into
    // runs of 16 consecutive rows of one column (128 contiguous bytes); lane
    // group gi = tid / 16 of the workgroup takes runs gi, gi + nthr/16, ...,
    // lane r = tid % 16 row r of each.  The workgroup has 4W lane groups
    // (W = ceil(Wn/16) waves) and X has 16W runs; G has 16 ceil(RT/2) runs
    // with RT <= ceil(2B/16) <= ceil(Wn/8) <= 2W (B <= Wn), so at most 16W
    // too: 4 runs of each per lane group.
    constexpr int kPG = 4, kPX = 4;
    const int gi = tid >> 4, r16 = tid & 15, ngrp = nthr >> 4;
    const int gruns = 16 * ((NO + 15) / 16), xruns = 16 * ((a.Wn + 15) / 16);
    float2 rgv[kPG], rxv[kPX];
    auto load = [&](int st) {
        const long long cb = col_lo + 16LL * st;
        const float2* gb = a.g + cb * a.N + (long long)b * a.B + o0;   // uniform
        const float2* xb = a.x + cb * a.N + s0;
#pragma unroll
        for (int u = 0; u < kPG; ++u) {
            const int pr = gi + u * ngrp, c = pr & 15, o = (pr >> 4) * 16 + r16;
            rgv[u] = (pr < gruns && o < NO && o0 + o < a.B && cb + c < col_hi)
                         ? gb[(unsigned)(c * a.N + o)] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kPX; ++u) {
            const int pr = gi + u * ngrp, c = pr & 15, j = (pr >> 4) * 16 + r16;
            rxv[u] = (pr < xruns && j < a.Wn && cb + c < col_hi)
                         ? xb[(unsigned)(c * a.N + j)] : make_float2(0.f, 0.f);
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < kPG; ++u) {
            const int pr = gi + u * ngrp, c = pr & 15, o = (pr >> 4) * 16 + r16;
            if (pr < gruns && o < NO) gT[o * kDwS + c] = rgv[u];
        }
#pragma unroll
        for (int u = 0; u < kPX; ++u) {
            const int pr = gi + u * ngrp, c = pr & 15, j = (pr >> 4) * 16 + r16;
            if (pr < xruns) xT[j * kDwS + c] = rxv[u];
        }
    };

    floatx4 acc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
    // window columns past Wn stay zero in xT: clear them once
    for (int e = tid; e < 16 * kDwMaxWaves * kDwS; e += nthr) xT[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const int jcol = wave * 16 + l16;   // this lane's window column (B operand)
    load(0);
    for (int st = 0; st < nsteps; ++st) {
        store();
        __syncthreads();
        if (st + 1 < nsteps) load(st + 1);
#pragma unroll
        for (int kg = 0; kg < 2; ++kg) {   // 8 columns = 16 reals = 4 k-steps each
            const int c = 8 * kg + 2 * q;  // this lane's two columns
            const float4 xv = *reinterpret_cast<const float4*>(&xT[jcol * kDwS + c]);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int r = rt * 16 + l16;
                const float4 gv = *reinterpret_cast<const float4*>(&gT[(r >> 1) * kDwS + c]);
                // real row 2o: (gr, gi) per column; row 2o+1: (gi, -gr)
                const float4 av = (r & 1) == 0 ? gv : make_float4(gv.y, -gv.x, gv.w, -gv.z);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bq(av, i), bq(xv, i), acc[rt], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    if (jcol >= a.Wn) return;
    float2* pp = a.part + ((long long)b * a.nch + ch) * a.B * (long long)a.Wn;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int o = o0 + ((rt * 16 + 4 * q) >> 1);
        const floatx4 v = acc[rt];
        if (o < a.B) pp[(long long)o * a.Wn + jcol] = make_float2(v[0], v[1]);
        if (o + 1 < a.B) pp[(long long)(o + 1) * a.Wn + jcol] = make_float2(v[2], v[3]);
    }
}

// dW_c[o][j] = sum over the blocks of class c and their column chunks of the
// FP32 partials, in FP64.  A workgroup takes 64 consecutive (c, o, j)
// entries; wave w sums the chunks ch = w mod 4 of every block of the class,
// and the four wave sums are added in a fixed order (deterministic).
__global__ __launch_bounds__(256) void dw_reduce_kernel(const float2* __restrict__ part,
                                                        const int* __restrict__ classes,
                                                        double2* __restrict__ dwc, int n_classes,
                                                        int nb, int nch, int B, int Wn) {
    __shared__ double2 red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long idx = (long long)blockIdx.x * 64 + lane;
    const long long per = (long long)B * Wn;
    double sx = 0.0, sy = 0.0;
    if (idx < per * n_classes) {
        const int c = (int)(idx / per);
        const long long e = idx % per;
        for (int b = 0; b < nb; ++b) {
            if (classes[b] != c) continue;
            const float2* p = part + (long long)b * nch * per + e;
#pragma unroll 4
            for (int ch = w; ch < nch; ch += 4) {
                const float2 v = p[(long long)ch * per];
                sx += v.x;
                sy += v.y;
            }
        }
    }
    red[w][lane] = make_double2(sx, sy);
    __syncthreads();
    if (w == 0 && idx < per * n_classes) {
        double2 t = red[0][lane];
        for (int k = 1; k < 4; ++k) {
            t.x += red[k][lane].x;
            t.y += red[k][lane].y;
        }
        dwc[idx] = t;
    }
}

// Z_c = dW_c A_c^-1.  A^-1 is Hermitian.  Stored column-major (the fixed
// design, one matrix for all classes, ainv_stride 0), A^-1[m][j] =
// conj(ainv[j + m Wn]); stored row-major (a caller correlation, one matrix
// per class), A^-1[m][j] = ainv[j + m Wn].  Consecutive j (threads) read
// consecutive entries, and the dW_c row is shared by the workgroup's threads.
__global__ void z_kernel(const double2* __restrict__ dwc, const double2* __restrict__ ainv,
                         double2* __restrict__ z, int n_classes, int B, int Wn,
                         long long ainv_stride, int rowmajor) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)B * Wn;
    if (idx >= per * n_classes) return;
    const long long row = idx / Wn;     // (c, o)
    const int j = (int)(idx % Wn);
    const double2* d = dwc + row * Wn;
    const double2* ai = ainv + (idx / per) * ainv_stride;
    const double cs = rowmajor ? -1.0 : 1.0;
    double sx = 0.0, sy = 0.0;
#pragma unroll 4
    for (int m = 0; m < Wn; ++m) {
        const double2 u = d[m], a = ai[j + (long long)m * Wn];
        const double2 v = make_double2(a.x, cs * a.y);   // conj(A^-1[m][j])
        sx += u.x * v.x + u.y * v.y;
        sy += u.y * v.x - u.x * v.y;
    }
    z[idx] = make_double2(sx, sy);
}

// Gamma_II[c][i][j] = -sum_o conj(W_c[o][i]) Z_c[o][j]
__global__ void gamma_kernel(const double2* __restrict__ w64, const double2* __restrict__ z,
                             double2* __restrict__ gam, int n_classes, int B, int Wn) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = (long long)Wn * Wn;
    if (idx >= per * n_classes) return;
    const int c = (int)(idx / per);
    const int i = (int)((idx % per) / Wn), j = (int)(idx % Wn);
    const double2* W = w64 + (long long)c * B * Wn;
    const double2* Z = z + (long long)c * B * Wn;
    double gx = 0.0, gy = 0.0;
#pragma unroll 4
    for (int o = 0; o < B; ++o) {
        const double2 w = W[(long long)o * Wn + i], zz = Z[(long long)o * Wn + j];
        gx -= w.x * zz.x + w.y * zz.y;
        gy -= w.x * zz.y - w.y * zz.x;
    }
    gam[idx] = make_double2(gx, gy);
}

// Per class: t1 = Re sum conj(Z) dR_OI, t2 = Re sum conj(Gamma_II) dR_II,
// t3 = Re tr(Gamma_II).  kPgSlices workgroups per class each reduce a fixed
// slice with a fixed-order tree; out[(c*kPgSlices + slice)*3 + 0..2].
constexpr int kPgSlices = 32;

__global__ __launch_bounds__(256) void param_grad_kernel(const double2* __restrict__ z,
                                                         const double2* __restrict__ gam,
                                                         const double2* __restrict__ rd,
                                                         const int* __restrict__ class_off,
                                                         double* __restrict__ out, int B, int Wn) {
    __shared__ double red[3][256];
    const int c = blockIdx.x / kPgSlices, sl = blockIdx.x % kPgSlices, tid = threadIdx.x;
    const double2* Z = z + (long long)c * B * Wn;
    const double2* G = gam + (long long)c * Wn * Wn;
    const double2* dr = rd + Wn;
    const int off = class_off[c];
    double t1 = 0.0, t2 = 0.0, t3 = 0.0;
    const int stride = 256 * kPgSlices;
    for (long long e = sl * 256 + tid; e < (long long)B * Wn; e += stride) {
        const int o = (int)(e / Wn), j = (int)(e % Wn);
        const int d = off + o - j;
        const double2 g = d >= 0 ? dr[d] : make_double2(dr[-d].x, -dr[-d].y);
        t1 += Z[e].x * g.x + Z[e].y * g.y;
    }
    for (long long e = sl * 256 + tid; e < (long long)Wn * Wn; e += stride) {
        const int i = (int)(e / Wn), j = (int)(e % Wn);
        const int d = i - j;
        const double2 g = d >= 0 ? dr[d] : make_double2(dr[-d].x, -dr[-d].y);
        t2 += G[e].x * g.x + G[e].y * g.y;
        if (i == j) t3 += G[e].x;
    }
    red[0][tid] = t1;
    red[1][tid] = t2;
    red[2][tid] = t3;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            for (int k = 0; k < 3; ++k) red[k][tid] += red[k][tid + s];
        __syncthreads();
    }
    if (tid == 0)
        for (int k = 0; k < 3; ++k) out[((long long)c * kPgSlices + sl) * 3 + k] = red[k][0];
}

// dscal[0] = dtau, dscal[1] = dlam, summed over classes and slices in order
__global__ void param_sum_kernel(const double* __restrict__ per, double* __restrict__ dscal,
                                 int n_classes) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double dt = 0.0, dl = 0.0;
    for (int c = 0; c < n_classes; ++c)
        for (int sl = 0; sl < kPgSlices; ++sl) {
            const double* q = per + ((long long)c * kPgSlices + sl) * 3;
            dt += q[0] + q[1];
            dl += q[2];
        }
    dscal[0] = dt;
    dscal[1] = dl;
}

// ---------------------------------------------------------------- host side
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int count_classes(const lmmse_plan_desc& d) {
    const int nb = d.N / d.B, halo = (d.Wn - d.B) / 2;
    if (d.rsource == LMMSE_R_USER_R) return nb;   // one filter per block
    std::vector<int> offs;
    for (int b = 0; b < nb; ++b) {
        const int s = std::min(std::max(b * d.B - halo, 0), d.N - d.Wn);
        const int o = b * d.B - s;
        if (std::find(offs.begin(), offs.end(), o) == offs.end()) offs.push_back(o);
    }
    return (int)offs.size();
}

// Workspace: W^H bank | dW partials | dW_c, Z_c | Gamma_II | per-class scalars
struct BwLayout {
    size_t bank, part, dwc, zc, gam, per, total;
};

static BwLayout bw_layout(const lmmse_plan_desc& d, int n_classes, const BwGeom& g) {
    BwLayout L{};
    const size_t bank = (size_t)n_classes * 2 * g.G16b * g.Rpad * 4 * sizeof(float4);   // 4 lanes q per row
    const size_t part = (size_t)(d.N / d.B) * g.nch * d.B * d.Wn * sizeof(float2);
    const size_t bw = (size_t)n_classes * d.B * d.Wn * sizeof(double2);
    const size_t gam = (size_t)n_classes * d.Wn * d.Wn * sizeof(double2);
    L.bank = 0;
    L.part = L.bank + align256(bank);
    L.dwc = L.part + align256(part);
    L.zc = L.dwc + align256(bw);
    L.gam = L.zc + align256(bw);
    L.per = L.gam + align256(gam);
    L.total = L.per + align256((size_t)n_classes * kPgSlices * 3 * sizeof(double));
    return L;
}

size_t backward_workspace_bytes(const lmmse_plan_desc& d, int slots) {
    if (d.rsource == LMMSE_R_SAMPLE)   // no sample backward above 256 (refused)
        return d.Wn > kMaxSampleWindowLarge ? 0 : sample_backward_workspace_bytes(d, slots);
    const long long ncols = (long long)slots * d.M * d.K;
    std::vector<int> starts;
    const int nb = d.N / d.B, halo = (d.Wn - d.B) / 2;
    for (int b = 0; b < nb; ++b) starts.push_back(std::min(std::max(b * d.B - halo, 0), d.N - d.Wn));
    const BwGeom g = bw_geom(d, starts, ncols);
    return bw_layout(d, count_classes(d), g).total;
}

// The parameter gradients of lmmse_backward on the device: out[0] = d_tau
// (EXPONENTIAL designs, else NaN), out[1] = d_sigma2 = dlam / K (not for
// caller filters: NaN), the host call's values and arithmetic.
__global__ void params_out_kernel(const double* __restrict__ dscal, double* __restrict__ out, int tau_ok,
                                  int sig_ok, double K) {
    out[0] = tau_ok ? dscal[0] : __builtin_nan("");
    out[1] = sig_ok ? dscal[1] / K : __builtin_nan("");
}

hipError_t launch_params_out(const Plan& p, double* out, hipStream_t st) {
    hipLaunchKernelGGL(params_out_kernel, dim3(1), dim3(1), 0, st, p.dscal, out,
                       p.d.rsource == LMMSE_R_EXPONENTIAL ? 1 : 0, p.d.rsource == LMMSE_R_USER ? 0 : 1,
                       (double)p.d.K);
    return hipGetLastError();
}

hipError_t launch_backward_fixed(Plan& p, int slots, const float2* hls, const float2* g,
                                 float2* dhls, bool want_params, void* ws, hipStream_t st) {
    const long long ncols = (long long)slots * p.d.M * p.d.K;
    if (ncols == 0) return hipSuccess;
    const int B = p.d.B, Wn = p.d.Wn, N = p.d.N;
    const BwGeom geo = bw_geom(p.d, p.h_starts, ncols);
    const BwLayout L = bw_layout(p.d, p.n_classes, geo);
    char* w = (char*)ws;
    float4* bank = (float4*)(w + L.bank);
    float2* part = (float2*)(w + L.part);
    double2* dwc = (double2*)(w + L.dwc);
    double2* zc = (double2*)(w + L.zc);
    double2* gam = (double2*)(w + L.gam);
    double* per = (double*)(w + L.per);
    // The design-gradient chain (dW partials -> per-class dW -> Z -> scalars)
    // reads nothing the dX passes write, so it runs on the plan's second
    // stream beside them, from a fork before the first dX launch to a join
    // after its last kernel.
    hipStream_t sd = st;
    if (want_params) {
        if (Wn > 16 * kDwMaxWaves) return hipErrorNotSupported;
        hipError_t e0 = hipEventRecord(p.fork, st);
        if (e0 == hipSuccess) e0 = hipStreamWaitEvent(p.side, p.fork, 0);
        if (e0 != hipSuccess) return e0;
        sd = p.side;
    }

    // W^H bank
    {
        const long long total = (long long)p.n_classes * 2 * geo.G16b * geo.Rpad * 4;
        hipLaunchKernelGGL(pack_wh_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                           p.w64, bank, p.n_classes, B, Wn, 2 * geo.G16b, geo.RT, geo.rgroups);
    }
    // One pass per window colour.  The first pass stores its windows; the
    // subcarriers none of them covers are zeroed before the later passes add
    // theirs (the whole of dX when there are too many such runs, and then
    // every pass adds).
    GapRuns gr{};
    {
        std::vector<char> cov(N, 0);
        for (int b = 0; b < p.nb; b += geo.P)
            for (int j = 0; j < Wn; ++j) cov[p.h_starts[b] + j] = 1;
        for (int n0 = 0; n0 < N && gr.n <= kMaxGapRuns; ++n0) {
            if (cov[n0] || (n0 > 0 && !cov[n0 - 1])) continue;
            int n1 = n0;
            while (n1 < N && !cov[n1]) ++n1;
            if (gr.n < kMaxGapRuns) {
                gr.lo[gr.n] = n0;
                gr.off[gr.n + 1] = gr.off[gr.n] + (n1 - n0);
            }
            ++gr.n;
        }
    }
    const bool store_first = gr.n <= kMaxGapRuns;
    if (!store_first) {
        const long long n = ncols * N;
        hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dhls, n);
    } else if (gr.n > 0) {
        const long long n = ncols * gr.off[gr.n];
        hipLaunchKernelGGL(fill_gaps_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dhls,
                           ncols, N, gr);
    }
    for (int pass = 0; pass < geo.P; ++pass) {
        const hipError_t e = launch_apply_f32_transposed(p, slots, bank, geo.RT, geo.rgroups, pass,
                                                         geo.P, g, dhls,
                                                         (pass == 0 && store_first) ? 0 : 1, st);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !want_params) return e;

    // dW partials -> per-class dW (FP64) -> Z -> scalars, on sd
    DwArgs dw;
    dw.starts = p.d_starts;
    dw.g = g;
    dw.x = hls;
    dw.part = part;
    dw.ncols = ncols;
    dw.cpw = geo.cpw;
    dw.N = N;
    dw.B = B;
    dw.Wn = Wn;
    dw.nb = p.nb;
    dw.nch = geo.nch;
    dw.rgroups = geo.dwRG;
    const dim3 gridw((unsigned)((long long)p.nb * geo.nch * geo.dwRG));
    const dim3 blockw(64 * ((Wn + 15) / 16));
    switch (geo.dwRT) {
#define LMMSE_DW(R) \
    case R: hipLaunchKernelGGL((dw_kernel<R>), gridw, blockw, 0, sd, dw); break;
        LMMSE_DW(1) LMMSE_DW(2) LMMSE_DW(3) LMMSE_DW(4) LMMSE_DW(5) LMMSE_DW(6) LMMSE_DW(7)
        LMMSE_DW(8) LMMSE_DW(9) LMMSE_DW(10) LMMSE_DW(11) LMMSE_DW(12) LMMSE_DW(13)
#undef LMMSE_DW
        default:
            return hipErrorInvalidValue;
    }
    const long long tot = (long long)p.n_classes * B * Wn;
    hipLaunchKernelGGL(dw_reduce_kernel, dim3((unsigned)((tot + 63) / 64)), dim3(256), 0, sd, part,
                       p.d_classes, dwc, p.n_classes, p.nb, geo.nch, B, Wn);
    const bool per_block = p.d.rsource == LMMSE_R_USER_R;
    hipLaunchKernelGGL(z_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, sd, dwc, p.ainv,
                       zc, p.n_classes, B, Wn, per_block ? (long long)Wn * Wn : 0LL, per_block ? 1 : 0);
    const long long totg = (long long)p.n_classes * Wn * Wn;
    hipLaunchKernelGGL(gamma_kernel, dim3((unsigned)((totg + 255) / 256)), dim3(256), 0, sd, p.w64, zc,
                       gam, p.n_classes, B, Wn);
    hipLaunchKernelGGL(param_grad_kernel, dim3(p.n_classes * kPgSlices), dim3(256), 0, sd, zc, gam,
                       p.rd, p.d_class_off, per, B, Wn);
    hipLaunchKernelGGL(param_sum_kernel, dim3(1), dim3(64), 0, sd, per, p.dscal, p.n_classes);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipEventRecord(p.join, sd);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, p.join, 0);
    return e;
}

}  // namespace lmmse
