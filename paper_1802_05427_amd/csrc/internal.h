// Internal declarations shared by the host API and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/lmmse.h"

namespace lmmse {

// Filter layouts the GEMM kernels read.  Wr is the 2B x 2Wn real embedding
// of a complex filter (rows 2a, 2a+1 = Re, Im of output a; columns 2j, 2j+1 =
// Re, Im of input j); its rows are padded to Rpad = RT*16*rgroups and split
// into rgroups row groups of RT*16 rows (one per workgroup).  Both banks are
// stored in the order a workgroup holds them in LDS, so that one chunk of one
// row group is a contiguous run:
//  * FP32 bank, groups g < 2*G16 of 8 complex window rows (16 reals), 4 lanes
//    q, rows rr of the row group:  bank[(((c*2*G16 + g)*rgroups + rg)*4 + q)
//    *RT*16 + rr] (float4) holds Wr[rg*RT*16 + rr][16g + 4q + i], i = 0..3.
//  * split banks, groups g < G16 of 16 complex rows (32 reals), 4 lanes kq:
//    part[((((c*G16 + g)*rgroups + rg)*4 + kq)*RT*16 + rr)*8 + e] holds the
//    part of Wr[rg*RT*16 + rr][32g + 8kq + e].
// Window rows past Wn and rows past 2B are zero.
struct Plan {
    lmmse_plan_desc d{};
    int device = 0;
    int nb = 0;          // number of blocks N/B
    int halo = 0;        // (Wn-B)/2
    int n_classes = 0;
    int RT = 0;          // 16-row MFMA tiles per workgroup row group
    int rgroups = 0;     // row groups per block: RT*16*rgroups = Rpad >= 2B
    int sRT = 0;         // the same for the split-precision filter of the sample path,
    int srgroups = 0;    // whose per-window filter parts take less LDS (up to 17 tiles)
    int Rpad = 0;        // padded real rows of a filter (RT*16*rgroups)
    int G8 = 0;          // ceil(Wn/8)
    int G16 = 0;         // ceil(Wn/16)
    std::vector<int> h_starts, h_offsets, h_classes, h_class_off;
    int* d_starts = nullptr;     // [nb]
    int* d_classes = nullptr;    // [nb]
    int* d_offsets = nullptr;    // [nb] output offset of each block in its window
    int* d_bstarts = nullptr;    // [nb] first output subcarrier of each block, b*B
    int* d_class_off = nullptr;  // [n_classes]
    double2* w64 = nullptr;      // [n_classes][B][Wn] FP64 filters
    double2* ainv = nullptr;     // [Wn][Wn] (R_II + lam I)^-1 of the fixed design (column-major);
                                 // caller correlation: [nb][Wn][Wn] per block (row-major)
    double2* rwin = nullptr;     // caller correlation: its windows R[I_b, I_b], [nb][Wn][Wn]
    double2* dwork = nullptr;    // caller correlation, Wn > 160: sweep scratch of nb windows
    double2* rd = nullptr;       // [3][Wn] r_d, dr_d/dtau (d = 0..Wn-1), x = A^-1 e_0
    float4* wf32 = nullptr;      // FP32 bank
    uint16_t* whi = nullptr;     // split bank, hi part
    uint16_t* wlo = nullptr;     // split bank, lo part (FP16: scaled by 2^11)
    float2* twiddle = nullptr;   // [K] exp(+j 2 pi r / K)
    int* status = nullptr;       // [2] device status word: code, info
    double* dscal = nullptr;     // [4] device scratch for the design backward
    // the fixed backward's design-gradient chain runs on `side` (default
    // priority) beside the dX passes: fork / join order it against the
    // caller's stream
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool ready = false;
    bool have_corr = false;      // caller correlation set (its windows in rwin)
    double design_sigma2 = 0.0;
    double design_tau = 0.0;
    float lo_scale = 1.0f;       // split-bank lo scale (FP16: 2^11)
    float in_scale = 1.0f;       // power-of-two scale of the LS values before a split
};

size_t fixed_bank_f32_elems(const Plan& p);    // float4 elements
size_t hls_bytes(const lmmse_plan_desc& d, int slots);   // H_LS staging, 256-byte multiple
size_t split_bank_elems(const Plan& p);        // uint16 elements per part
// Workspace lmmse_estimate needs for `slots` slots (0 on the fused fixed path).
size_t forward_workspace_bytes(const lmmse_plan_desc& d, int slots);
// Device a plan was created on.
int plan_device(lmmse_plan_t plan);

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_despread(const Plan& p, int slots, const float2* y, const float2* pilots,
                           float2* hls, hipStream_t st);
hipError_t launch_apply_f32(const Plan& p, int slots, const float2* x, const float2* pilots,
                            bool fused, float2* out, hipStream_t st);
hipError_t launch_apply_split(const Plan& p, int slots, const float2* x, const float2* pilots,
                              bool fused, float2* out, hipStream_t st);
bool apply_fusable(const Plan& p);
// The FP32 filtering kernel with transposed roles (backward dX): for blocks
// pass, pass + P, ..., dx[col][start_b + i] += sum_o Wr^H[i][o] g[col][bB + o],
// i < Wn, with `bank` the real embedding of W^H (2Wn x 2B) laid out as the
// FP32 bank (RT-row tiles, rgroups row groups, ceil(B/16) chunks).
void transposed_row_tiles(int out_len, int& RT, int& rgroups);
hipError_t launch_apply_f32_transposed(const Plan& p, int slots, const float4* bank, int RT,
                                       int rgroups, int pass, int P, const float2* g, float2* dx,
                                       int accumulate, hipStream_t st);

// Fixed design: r_d (and d r_d / d tau) on the device, A^-1 of the Toeplitz
// A = R_II + lam I, then class filters W_c = (I - lam A^-1)[off_c rows].
hipError_t launch_fixed_design(Plan& p, double tau, double sigma2, hipStream_t st);
// Convert p.w64 into the FP32 and split banks.
hipError_t launch_pack_banks(Plan& p, hipStream_t st);

// Sample-covariance path.
hipError_t launch_covariance(const Plan& p, int slots, const float2* hls, double2* r_win,
                             hipStream_t st);
// Register-resident design (Wn <= 160) from window correlations r_win
// [nmat][Wn][Wn] (row-major): W [nmat][B][Wn] with offsets[mat % nb] and,
// when ainv is not null, A^-1 = (R + lam I)^-1 [nmat][Wn][Wn] (row-major).
hipError_t launch_batched_filters(const Plan& p, long long nmat, const double2* r_win, double lam,
                                  double2* w_out, double2* ainv, hipStream_t st);
// keep_w64 / keep_ainv (both or neither; windows resident_design_fits):
// each window's FP64 filter rows [nmat][B][Wn] and (R + lam I)^-1
// [nmat][Wn][Wn] as well, for a backward that does not redesign.
hipError_t launch_sample_estimate(const Plan& p, int slots, const float2* hls, double lam,
                                  float2* out, void* ws, hipStream_t st,
                                  double2* keep_w64 = nullptr, double2* keep_ainv = nullptr);
size_t sample_workspace_bytes(const lmmse_plan_desc& d, int slots);
// Per (slot, user, block) window of the sample design: W (FP64 [nmat][B][Wn])
// and A^-1 = (R + lam I)^-1 (FP64 [nmat][Wn][Wn], both triangles); scratch:
// sweep_scratch_bytes(Wn, nmat), used by windows wider than the register
// sweep.
hipError_t launch_sample_inverse(const Plan& p, long long nmat, long long mat0, const float2* hls,
                                 double lam, double2* w64, double2* ainv, double2* scratch,
                                 hipStream_t st);
size_t sample_backward_workspace_bytes(const lmmse_plan_desc& d, int slots);
// Windows the register-resident sample design holds, and the limit of the
// workspace-resident one (sample_large.hip) used above it.
constexpr int kMaxSampleWindowReg = 160;
constexpr int kMaxSampleWindowLarge = 256;
// Sample designs of windows wider than this (up to 208) run in the resident
// kernel (resident_inverse.hip), narrower ones in sample.hip.
constexpr int kResidentFp64Cov = 128;
constexpr int kSweepPanel = 64;   // pivots per panel of the workspace-resident sweep
// Windows wider than kMaxSampleWindowLarge: the push-through form (M x M
// systems), for up to this many antennas.
constexpr int kMaxPushthroughAntennas = 256;
// -(A + lam I)^-1 in place for nmat Hermitian n x n matrices [mat][n][n]
// (both triangles), batch index (slot * K + user) * nb + block; scratch:
// sweep_scratch_bytes(n, nmat).  Non-positive pivot: LMMSE_ERR_NOT_PD with
// matrix mat0 + mat in status.
hipError_t launch_sweep_inverse(long long nmat, long long mat0, int n, int K, int nb, double lam,
                                double2* amat, double2* scratch, int* status, hipStream_t st);
// The same for n <= 208 with one workgroup holding a whole matrix (no
// scratch); resident_inverse_fits(n) says whether it applies.
bool resident_inverse_fits(int n);
hipError_t launch_resident_inverse(long long nmat, long long mat0, int n, double lam, double2* amat,
                                   int* status, hipStream_t st);
// The sample design of windows 129..208 wide in the same kernel
// (resident_design_fits): R = X X^H / M from the LS values (FP64 products and
// sums up to 160, FP32 ones as the batched product above), its
// inverse, and the block filters W = (I - lam A^-1)[off_b rows] into any of
// w64 / w32 / whi, wlo (the layouts of launch_sample_large); with want_ainv
// A^-1 into amat [nmat][Wn][Wn] (otherwise amat is not touched).  Matrix
// indices as in launch_sample_large (hls and nmat of one chunk of slots).
bool resident_design_fits(int Wn);
hipError_t launch_resident_design(const Plan& p, long long nmat, long long mat0, const float2* hls, double lam,
                                  double2* amat, double2* w64, float2* w32, uint32_t* whi, uint32_t* wlo,
                                  bool want_ainv, hipStream_t st);
// From S = -(R + lam I)^-1 as launch_sweep_inverse leaves it, the block
// filters W = (I + lam S)[off_b rows] (w64 [mat][B][Wn]; offsets indexed by
// mat % nb) and, with negate, A^-1 = -S in place.
hipError_t launch_large_filters(long long nmat, double2* amat, const int* offsets, int B, int Wn,
                                int nb, double lam, double2* w64, bool negate, hipStream_t st);
// Push-through estimate of windows wider than kMaxSampleWindowLarge: work
// area pushthrough_bytes(d, nmat) = amat [nmat][M][M] then sweep scratch.
size_t pushthrough_bytes(const lmmse_plan_desc& d, long long nmat);
hipError_t launch_sample_pushthrough(const Plan& p, long long nmat, long long mat0, const float2* hls,
                                     double lam, double2* amat, double2* scratch, float2* out,
                                     hipStream_t st);
// Caller correlation (LMMSE_R_USER_R): windows of the N x N matrix into
// p.rwin, then the block filters from p.rwin at lam = sigma2 / K.
hipError_t launch_user_corr_gather(Plan& p, const double2* r, hipStream_t st);
hipError_t launch_user_corr_design(Plan& p, double sigma2, hipStream_t st);
size_t user_corr_scratch_bytes(const lmmse_plan_desc& d);
// Workspace-resident sample design of nmat windows: amat [nmat][Wn][Wn] and
// scratch (sweep_scratch_bytes) are device work areas; w64 / w32 / whi, wlo
// may be null; with want_ainv amat ends as A^-1.
size_t large_design_bytes(const lmmse_plan_desc& d, long long nmat);
size_t sweep_scratch_bytes(int Wn, long long nmat);   // the scratch part of it
hipError_t launch_sample_large(const Plan& p, long long nmat, long long mat0, const float2* hls,
                               double lam, double2* amat, double2* scratch, double2* w64,
                               float2* w32, uint32_t* whi, uint32_t* wlo, bool want_ainv,
                               hipStream_t st);
// Split-precision filtering of the sample path with per-window filter parts
// whi / wlo [mat][B][Wq] (Wq = Wn rounded up to 4).
hipError_t launch_apply_sample_split(const Plan& p, long long nmat, const float2* hls,
                                     const uint32_t* whi, const uint32_t* wlo, float2* out,
                                     hipStream_t st);
hipError_t launch_covariance_large(const Plan& p, long long nmat, const float2* hls, double2* r_win,
                                   hipStream_t st);

// Backward.
size_t backward_workspace_bytes(const lmmse_plan_desc& d, int slots);
hipError_t launch_backward_fixed(Plan& p, int slots, const float2* hls, const float2* g,
                                 float2* dhls, bool want_params, void* ws, hipStream_t st);
// d_tau, d_sigma2 of the last backward into device out[2] (lmmse_backward_dev).
hipError_t launch_params_out(const Plan& p, double* out, hipStream_t st);
// kept_w64 / kept_ainv: the design of launch_sample_estimate's keep buffers
// for the same h_ls and lam (not recomputed); null: designed again here.
hipError_t launch_backward_sample(Plan& p, int slots, const float2* hls, const float2* g,
                                  float2* dhls, double lam, bool want_sigma, void* ws,
                                  hipStream_t st, const double2* kept_w64 = nullptr,
                                  const double2* kept_ainv = nullptr);

}  // namespace lmmse
