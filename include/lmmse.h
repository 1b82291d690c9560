/*
 * lmmse.h - C ABI of the partitioned LMMSE channel estimator for gfx950.
 *
 * The estimator follows Sec. IV of the paper: least-squares estimates at the
 * pilots (eq. 8-9), an LMMSE weighting of them (eq. 12) with the weight of
 * eq. 13 / eq. 17 computed from a subcarrier correlation (eq. 14-16), and the
 * dimension reduction of Sec. IV-B that partitions the N x N correlation into
 * small blocks with overlapping or non-overlapping input windows
 * (Tables I-II).
 *
 * Problem layout (all device buffers are caller-owned, complex numbers are
 * interleaved (re, im), subcarrier index fastest):
 *   y_pilot  complex64 [S][M][K][N]  received pilot symbols: slot s, antenna m,
 *                                    pilot OFDM symbol t (K of them), subcarrier n
 *   pilots   complex64 [K][N]        unit-modulus pilot x_k[n] of user k
 *   h_ls     complex64 [S][M][K][N]  LS estimate (user k third)
 *   h_hat    complex64 [S][M][K][N]  LMMSE estimate
 * User k sends c[k,t] x_k[n] on pilot symbol t, c[k,t] = exp(-j 2 pi k t / K)
 * (a K x K DFT cover code), so LS despreading is
 *   h_ls[s,m,k,n] = conj(x_k[n]) (1/K) sum_t conj(c[k,t]) y[s,m,t,n]
 * and the LS noise variance is lam = sigma2 / K, which the filters use where
 * eq. 13 writes sigma^2 / sigma_s^2.
 *
 * Block plan: output block b = subcarriers [b*B, (b+1)*B) is estimated from
 * the window [start_b, start_b + Wn) with
 *   start_b = clamp(b*B - (Wn-B)/2, 0, N - Wn)
 * i.e. the window is centred on its block and shifted (never truncated) at
 * the band edges, as in Tables I-II.  Wn == B is the non-overlapping
 * partition, B == Wn == N the full-band LMMSE of eq. 13.  Requirements:
 * N % B == 0, (Wn - B) even, B <= Wn <= N.
 *
 * Correlation sources:
 *   LMMSE_R_UNIFORM      fixed design of eq. 16 with assumed channel length L
 *                        (in samples, relative to N_fft):
 *                        r_d = (1 - exp(-j2 pi L d/N_fft)) / (j2 pi L d/N_fft)
 *   LMMSE_R_EXPONENTIAL  fixed design from the exponential power-delay
 *                        profile of Sec. IV-A on integer taps l < taps:
 *                        r_d = sum_l p_l exp(-j2 pi l d/N_fft), p_l ~ e^{-l/tau}
 *   LMMSE_R_SAMPLE       raw sample covariance over the M antennas, per
 *                        (slot, user, window): R = (1/M) sum_m h h^H;
 *                        windows up to 256 are designed directly (up to 160
 *                        held in registers, R summed in FP64; wider ones in
 *                        the workspace, R summed in FP32 on the matrix
 *                        cores);
 *                        wider windows, e.g. the full band B = Wn = N, use
 *                        the equal push-through form W X = X_O G (G + lam I)^-1
 *                        with the M x M Gram matrix G = X^H X / M of the
 *                        window (M <= 256, FP32 precision only)
 *   LMMSE_R_USER         filters supplied by the caller (lmmse_set_filters);
 *                        also named LMMSE_R_USER_W
 *   LMMSE_R_USER_R       an N x N subcarrier correlation R_HH supplied by the
 *                        caller (lmmse_set_correlation), from which the plan
 *                        designs every block's filter on the device in FP64;
 *                        R need not be Toeplitz, so every block is its own
 *                        class (N/B filters)
 * For a fixed design every block whose window sits at the same offset
 * start_b - b*B shares one filter ("class"); there are at most 3 classes
 * when the halo (Wn-B)/2 is at most B (first, interior, last block).
 *
 * Precision: filters are designed in FP64.  A fixed design's R_II + lam I is
 * Hermitian Toeplitz and is inverted in O(Wn^2) (Levinson-Durbin recursion,
 * then the Gohberg-Semencul formula); the sample design inverts each window
 * matrix by a Hermitian sweep (Gauss-Jordan on the lower triangle).  Since
 * W = R_OI (R_II + lam I)^-1 = [I - lam (R_II + lam I)^-1] restricted to the
 * kept rows, the inverse alone gives the filter.  The filtering GEMM runs
 * in FP32 on the matrix cores (LMMSE_FP32), or as split products
 * hi*hi + hi*lo + lo*hi with FP32 accumulation in BF16 (LMMSE_BF16X3) or
 * FP16 (LMMSE_FP16X3); the sample-covariance path writes each window's
 * filter as hi / lo parts and filters with the same split products.
 * FP16X3 range: the filtering kernels split s * h_ls, s the plan's
 * power-of-two input scale (lmmse_set_input_scale, default 1), and undo s on
 * the output (both exact); |s h_ls| must stay below 65504 and every filter
 * entry below 32 (LMMSE filters are below 1; caller filters are checked).
 * A value past either limit records LMMSE_ERR_RANGE (info -1) for
 * lmmse_sync_status, and the affected outputs are not finite.  Below about
 * 1.2e-4 the FP16 lo part turns subnormal and the split loses accuracy
 * gradually, so s should bring the LS values to order one.  BF16X3 has the
 * FP32 range; FP32 results do not depend on s.
 * The backward products are FP32 on the matrix cores (fixed designs), or
 * FP64 and FP32 batched products on the matrix cores (sample covariance).
 *
 * Calls with slots == 0 launch nothing and accept NULL data pointers.
 *
 * Errors: every call returns an lmmse_status.  No exception crosses the ABI.
 * Device-side conditions (a non-positive pivot in a factorisation) are
 * recorded in a plan-owned status word, read by lmmse_sync_status.
 * Threading: a plan is not thread-safe; distinct plans are independent.
 * Streams: kernels run on the stream passed in (a hipStream_t, 0 = default
 * stream); calls return without synchronising unless stated.
 */
#ifndef LMMSE_H
#define LMMSE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lmmse_status {
    LMMSE_OK = 0,
    LMMSE_ERR_INVALID_ARG = 1,   /* null pointer, bad size, bad enum         */
    LMMSE_ERR_UNSUPPORTED = 2,   /* plan shape the library does not handle   */
    LMMSE_ERR_WORKSPACE = 3,     /* workspace missing or too small           */
    LMMSE_ERR_HIP = 4,           /* a HIP runtime call failed                */
    LMMSE_ERR_NOT_PD = 5,        /* R_II + lam I not positive definite       */
    LMMSE_ERR_NOT_READY = 6,     /* no filters designed or set yet           */
    LMMSE_ERR_NO_DEVICE = 7,     /* no usable gfx950 device                  */
    LMMSE_ERR_RANGE = 8          /* a value outside the FP16 split range     */
} lmmse_status;

typedef enum lmmse_rsource {
    LMMSE_R_UNIFORM = 0,
    LMMSE_R_EXPONENTIAL = 1,
    LMMSE_R_SAMPLE = 2,
    LMMSE_R_USER = 3,
    LMMSE_R_USER_R = 4
} lmmse_rsource;
#define LMMSE_R_USER_W LMMSE_R_USER

typedef enum lmmse_precision {
    LMMSE_FP32 = 0,
    LMMSE_BF16X3 = 1,
    LMMSE_FP16X3 = 2
} lmmse_precision;

/* Plan descriptor.  Sizes are counts; tau_rms and L are in samples. */
typedef struct lmmse_plan_desc {
    int M;           /* BS antennas                                  (>= 1) */
    int K;           /* users = pilot OFDM symbols                   (1..64) */
    int N;           /* used subcarriers                                    */
    int N_fft;       /* FFT size (>= N)                                     */
    int B;           /* output block size                                   */
    int Wn;          /* input window size                                   */
    int rsource;     /* lmmse_rsource                                       */
    int precision;   /* lmmse_precision                                     */
    int max_slots;   /* largest S any call on this plan will pass  (>= 1;
                        max_slots * M * K * N < 2^32 coefficients, as
                        per-coefficient kernels run one work-item each)   */
    int taps;        /* LMMSE_R_EXPONENTIAL: number of integer taps (>= 1)   */
    double tau_rms;  /* LMMSE_R_EXPONENTIAL: profile decay (> 0)            */
    double L;        /* LMMSE_R_UNIFORM: assumed channel length (> 0)       */
    double sigma2;   /* design noise variance per resource element (> 0)    */
} lmmse_plan_desc;

typedef struct lmmse_plan *lmmse_plan_t;

/* ---- host-only calls (no device needed) -------------------------------- */

/* Static text for a status code; never NULL. */
const char *lmmse_status_string(int status);

/* ABI version: major * 10000 + minor * 100 + patch. */
int lmmse_version(void);

/* Checks a descriptor without touching a device.  Returns LMMSE_OK,
 * LMMSE_ERR_INVALID_ARG (nonsensical values) or LMMSE_ERR_UNSUPPORTED. */
int lmmse_plan_validate(const lmmse_plan_desc *desc);

/* Block plan of Sec. IV-B (see top of file).  starts and offsets receive
 * N/B ints each, classes N/B ints with the filter class of every block;
 * *n_classes receives the number of distinct window offsets.  Any output
 * pointer may be NULL.  Host memory. */
int lmmse_block_plan(int N, int B, int Wn, int *starts, int *offsets,
                     int *classes, int *n_classes);

/* Workspace bytes lmmse_estimate / lmmse_backward need for `slots` slots
 * (0 for paths that need none).  Host memory output. */
int lmmse_workspace_size(const lmmse_plan_desc *desc, int slots, size_t *bytes);

/* ---- plan lifetime ------------------------------------------------------ */

/* Validates desc, allocates the plan's device buffers (filter bank, FP64
 * factors, status word) on the current device and, for the fixed designs,
 * builds the filters from desc (synchronously).  *out is set only on
 * success.  Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, HIP, NOT_PD. */
int lmmse_plan_create(const lmmse_plan_desc *desc, lmmse_plan_t *out);

/* Frees the plan and its device memory (synchronises the device first). */
int lmmse_plan_destroy(lmmse_plan_t plan);

/* Copies the descriptor the plan was created with (tau_rms / sigma2 updated
 * by the last lmmse_set_design). */
int lmmse_plan_get_desc(lmmse_plan_t plan, lmmse_plan_desc *out);

/* ---- filter design (eq. 13 / eq. 17 per block, FP64) --------------------- */

/* Rebuilds a fixed design (UNIFORM or EXPONENTIAL) with a new tau_rms
 * (EXPONENTIAL only; ignored for UNIFORM) and design noise sigma2, on
 * `stream`: r_d, then per class the inverse of A = R_II + lam I
 * (Levinson-Durbin + Gohberg-Semencul), W = I - lam A^-1 on the kept rows,
 * then the FP32 / split copies.  Asynchronous.  A non-positive prediction
 * error (A not positive definite) is reported by lmmse_sync_status. */
int lmmse_set_design(lmmse_plan_t plan, double tau_rms, double sigma2, void *stream);
/* On a SAMPLE plan it only records sigma2 (tau_rms ignored, nothing is
 * launched): the noise variance lmmse_backward differentiates at.  On a
 * USER_R plan it records sigma2 and, once a correlation has been set,
 * redesigns the filters from it (tau_rms ignored). */

/* Installs caller filters (LMMSE_R_USER plans): w is device complex128
 * [n_classes][B][Wn], row-major per filter, class order as lmmse_block_plan
 * numbers them.  Asynchronous (reads w on `stream`). */
int lmmse_set_filters(lmmse_plan_t plan, const void *w, void *stream);

/* Caller correlation (LMMSE_R_USER_R plans; eq. 13 with R_HH given, per
 * block of Sec. IV-B): r is device complex128 [N][N], row-major, Hermitian
 * (both triangles are read as given) and positive semi-definite.  The plan
 * copies the windows R[I_b, I_b] out of it (r may be freed after the stream
 * reaches this call) and designs W_b = R[O_b, I_b] (R[I_b, I_b] + lam I)^-1,
 * lam = sigma2 / K at the plan's design sigma2, for every block b (class b)
 * on `stream`: the register-resident Hermitian sweep up to Wn = 160, the
 * panel sweep above.  Asynchronous; a non-positive pivot is reported by
 * lmmse_sync_status (info = block).  Errors: INVALID_ARG, UNSUPPORTED (not a
 * USER_R plan), HIP. */
int lmmse_set_correlation(lmmse_plan_t plan, const void *r, void *stream);

/* Power-of-two scale s of the LS values inside the split-precision
 * filtering (see Precision above): the kernels split s * h_ls and multiply
 * the output by 1/s, so the estimate is unchanged while its FP16 parts stay
 * in range.  s = 2^e with -59 <= e <= 61, else INVALID_ARG.  Host only;
 * applies to the launches that follow. */
int lmmse_set_input_scale(lmmse_plan_t plan, double scale);

/* Copies the current FP64 filters of a fixed-design or user plan to device
 * complex128 [n_classes][B][Wn] (n_classes = N/B for USER_R).  Asynchronous. */
int lmmse_get_filters(lmmse_plan_t plan, void *w_out, void *stream);

/* ---- forward path ------------------------------------------------------- */

/* LS despreading only (eq. 8-9 with the cover code): y_pilot -> h_ls. */
int lmmse_despread(lmmse_plan_t plan, int slots, const void *y_pilot,
                   const void *pilots, void *h_ls, void *stream);

/* Filtering only (eq. 12 per block) with the plan's fixed or user filters:
 * h_ls -> h_hat, at the plan's precision. */
int lmmse_apply(lmmse_plan_t plan, int slots, const void *h_ls, void *h_hat,
                void *stream);

/* Sample covariance per (slot, user, window), R = (1/M) sum_m h_m h_m^H over
 * the antennas (not a step of the paper: the data-driven R that eq. 13 takes
 * as given, estimated from the LS values of the M antennas), products of
 * the complex64 LS values accumulated in FP64 (the estimate itself sums the
 * covariance of windows wider than 160 in FP32), stored as complex128
 * [S][K][N/B][Wn][Wn] (full matrix, both triangles).  Any plan. */
int lmmse_covariance(lmmse_plan_t plan, int slots, const void *h_ls,
                     void *r_win, void *stream);

/* Batched FP64 block filters from window correlations r_win (complex128
 * [S][K][N/B][Wn][Wn], e.g. from lmmse_covariance): for block b,
 * W = R[off_b : off_b + B, :] (R + (sigma2/K) I)^-1, stored as complex128
 * [S][K][N/B][B][Wn].  Windows up to 160 use the register-resident sweep
 * and no workspace; wider windows copy r_win into ws and invert there by the
 * panel sweep (ws: lmmse_sample_filters_workspace_size bytes, else
 * LMMSE_ERR_WORKSPACE).  r_win is not modified. */
int lmmse_sample_filters_workspace_size(const lmmse_plan_desc *desc, int slots,
                                        size_t *bytes);
int lmmse_sample_filters(lmmse_plan_t plan, int slots, const void *r_win,
                         double sigma2, void *w_out, void *ws, size_t ws_bytes,
                         void *stream);

/* The whole estimator, estimate(y_pilot, pilots, sigma2, block plan) -> h_hat.
 * Fixed/user designs: a fused despread + filter launch with the plan's
 * filters (redesigned first if sigma2 differs from the design's).
 * Sample covariance: despread, covariance, FP64 block design with lam =
 * sigma2 / K, filter.  ws: device workspace of lmmse_workspace_size bytes
 * (may be NULL when that size is 0). */
int lmmse_estimate(lmmse_plan_t plan, int slots, const void *y_pilot,
                   const void *pilots, double sigma2, void *h_hat,
                   void *ws, size_t ws_bytes, void *stream);

/* The estimator from LS estimates, h_ls -> h_hat (lmmse_estimate without the
 * despreading): fixed and user designs filter with the plan's filters
 * (a fixed design is rebuilt first if sigma2 differs from its own); a
 * sample-covariance plan forms each window's covariance from h_ls, designs
 * with lam = sigma2 / K and filters.  Records sigma2 as the plan's design
 * noise (the value lmmse_backward uses on a sample plan).  ws as for
 * lmmse_estimate (sample plans; may be NULL otherwise).  This is the
 * function whose gradients lmmse_backward returns. */
int lmmse_estimate_ls(lmmse_plan_t plan, int slots, const void *h_ls,
                      double sigma2, void *h_hat, void *ws, size_t ws_bytes,
                      void *stream);

/* ---- backward path ------------------------------------------------------- */

/* Gradients of a real loss through lmmse_estimate_ls, given g =
 * dL/dRe(h_hat) + j dL/dIm(h_hat) (complex64 [S][M][K][N]).  Writes d_hls
 * (same layout) and, when the pointers are non-NULL, the host doubles *d_tau
 * (EXPONENTIAL design only; NaN otherwise) and *d_sigma2 (fixed and sample
 * designs); requesting them synchronises `stream`.
 * Fixed designs: d_hls = sum_b W_b^H g_b (overlapping windows add), and the
 * design parameters by implicit differentiation of the block solve.
 * Sample covariance (at the sigma2 of the last lmmse_estimate_ls /
 * lmmse_estimate / lmmse_set_design): per (slot, user, window) the filter
 * depends on h_ls through R as well, so d_hls also receives
 * (Gam + Gam^H) X / M with Gam the window's gradient of R (the gradient
 * of the FP64 design, whatever the filtering precision).  USER_R: d_hls
 * and *d_sigma2 (per-block inverses); *d_tau is NaN.  USER (caller
 * filters): d_hls only.  Windows wider than 256: d_hls only, for fixed,
 * USER_R and USER plans; requesting d_tau / d_sigma2 there, or any sample
 * backward, returns LMMSE_ERR_UNSUPPORTED before anything is launched.  ws:
 * lmmse_workspace_size bytes.  The design-parameter gradients of a fixed
 * design run on a stream the plan owns, beside the d_hls passes, ordered
 * after the work already on `stream` and before the work queued on it after
 * the call (event fork and join; graph capture of `stream` takes both). */
int lmmse_backward(lmmse_plan_t plan, int slots, const void *h_ls,
                   const void *g, void *d_hls, double *d_tau, double *d_sigma2,
                   void *ws, size_t ws_bytes, void *stream);

/* The same backward (the implicit differentiation of the eq. 13 / eq. 17
 * block solves, Sec. IV-B) with the design-parameter gradients left on the
 * device, for training loops that keep tau_rms and sigma2 on the GPU: no
 * step waits for the host.  d_params, when not NULL, is device memory of
 * two doubles written on `stream` after the backward's kernels:
 * d_params[0] = d_tau and d_params[1] = d_sigma2, with the values and NaNs
 * lmmse_backward returns.  Nothing is synchronised; d_params is the
 * caller's.  Arguments and errors otherwise as lmmse_backward (d_params
 * takes the place of requesting both scalars). */
int lmmse_backward_dev(lmmse_plan_t plan, int slots, const void *h_ls,
                       const void *g, void *d_hls, void *d_params,
                       void *ws, size_t ws_bytes, void *stream);

/* ---- sample design kept for the backward ---------------------------------- */

/* Bytes of the design a sample-covariance forward can keep for its backward
 * (eq. 13 per (slot, user, window), Sec. IV-B): for `slots` slots, each
 * window's FP64 filter rows W (B x Wn) and (R + lam I)^-1 (Wn x Wn), complex
 * doubles, [nmat][B][Wn] then [nmat][Wn][Wn] with nmat = slots * K * N / B
 * (1.05 MB per window at B = 132, Wn = 198).  *bytes is 0 where the plan
 * cannot keep it: not a sample plan, or windows outside 129..208 (the
 * designs held by one compute unit).  LMMSE_ERR_INVALID_ARG for a NULL plan
 * or bytes, or slots outside 0..max_slots. */
int lmmse_design_state_size(lmmse_plan_t plan, int slots, size_t *bytes);

/* lmmse_estimate_ls on a sample plan that also writes each window's FP64
 * filter rows and inverse into `state` (device memory of
 * lmmse_design_state_size bytes, the caller's), in the same launch and with
 * the same arithmetic as the design lmmse_backward recomputes; h_hat is
 * bit-identical to lmmse_estimate_ls's.  LMMSE_ERR_UNSUPPORTED where
 * lmmse_design_state_size gives 0, LMMSE_ERR_WORKSPACE for a short state or
 * ws (ws as for lmmse_estimate_ls). */
int lmmse_estimate_ls_keep(lmmse_plan_t plan, int slots, const void *h_ls,
                           double sigma2, void *h_hat, void *state,
                           size_t state_bytes, void *ws, size_t ws_bytes,
                           void *stream);

/* lmmse_backward_dev on a sample plan with the design read from `state`
 * instead of formed again: for training loops that run the forward and then
 * the backward of the same batch.  The state must come from
 * lmmse_estimate_ls_keep with the same slots and h_ls, and the plan's design
 * sigma2 must not have changed since (the caller's contract: nothing checks
 * it, and another h_ls gives the gradient of another estimate).  The state
 * is only read, so several backward calls may use it.  Results are
 * bit-identical to lmmse_backward_dev's.  Errors as lmmse_estimate_ls_keep
 * and lmmse_backward_dev. */
int lmmse_backward_kept(lmmse_plan_t plan, int slots, const void *h_ls,
                        const void *g, void *d_hls, void *d_params,
                        const void *state, size_t state_bytes, void *ws,
                        size_t ws_bytes, void *stream);

/* ---- estimate without a workspace argument ------------------------------- */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * estimate of lmmse_estimate with the library's own static device workspace
 * of LMMSE_NOALLOC_SCRATCH_BYTES instead of a caller buffer.  The caller
 * still passes the inputs and the output.  Nothing is allocated or freed:
 * the workspace is a file-scope device array, which every GPU the library
 * runs on holds until the process ends, and whose address is looked up once
 * per device (the first call on a device).  Every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (on other streams or other
 * threads) race; the array keeps the last call's contents, and nothing is
 * read from it before being written.  The plan's device must be current
 * (else INVALID_ARG).  Returns LMMSE_ERR_WORKSPACE, launching nothing, when
 * the estimate needs more than LMMSE_NOALLOC_SCRATCH_BYTES (lmmse_workspace_size
 * of the forward path: 0 for the fused fixed designs, H_LS staging for
 * unfused user counts, H_LS and the per-window filters for the sample
 * covariance).  Otherwise as lmmse_estimate. */
#define LMMSE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int lmmse_estimate_noalloc(lmmse_plan_t plan, int slots, const void *y_pilot,
                           const void *pilots, double sigma2, void *h_hat,
                           void *stream);

/* ---- status ------------------------------------------------------------- */

/* Synchronises `stream`, returns LMMSE_OK or the first device-detected error
 * since the last call (then clears it); *info (may be NULL) receives the
 * index of the failing matrix (slot * K * N/B + user * N/B + block for the
 * sample path, the class for fixed designs) or -1. */
int lmmse_sync_status(lmmse_plan_t plan, void *stream, int *info);

/* ---- comb-pilot 3W / 12W estimators (Sec. IV-B, Tables I-II) ------------- */

/* The paper's own partitioned estimators for comb pilots.  One pilot OFDM
 * symbol carries the pilot of UE k (0-based) on the comb tones k, k + S,
 * k + 2S, ... (S = comb spacing, N / S tones; eq. 6), so
 *   y[slot][m][n] = H_k[n] x[n] + w,  k = n mod S,
 * and the LS value of UE k on its tone t is y[t] / x[t] (eq. 9).  Group b of
 * a UE (one per tone) filters the `win` consecutive tones starting at
 *   wst_b = clamp(b - (win - 1) / 2, 0, N/S - win)
 * (win = 3 for 3W, 12 for 12W; Tables I and II) with
 *   W_b = R_OI (R_II + sigma2 I)^-1,  R[a][c] = r(a - c)
 * (eq. 13 / eq. 17 with a unit-modulus pilot: sigma_s^2 = 1; the 3W weights
 * W(1..3) with P read as the inverse), r from eq. 16 (UNIFORM, length L) or
 * the exponential tap sum (EXPONENTIAL).  Outputs of group b:
 *   LMMSE_COMB_3W:  subcarriers k + S b + j S/3, j = 0..2 (those below N),
 *                   and every subcarrier without an estimate takes the
 *                   latest estimate below it (zero-order hold, Sec. IV-C),
 *                   the first estimate below the first one;
 *   LMMSE_COMB_12W: the S subcarriers S b .. S b + S - 1.
 * W_b depends only on b - wst_b (and, for 12W, on k): each UE has `win`
 * filter classes, designed in FP64 on the device when the plan is made and
 * applied in FP32.  The interpolated-LS baselines (Sec. IV-A-1: LS_HOLD,
 * LS_LINEAR, LS_LINEAR3, LS_QUADRATIC, LS_SPLINE) use the same LS values and
 * no filters (get_filters returns zeros); all run in FP32. */
typedef enum lmmse_comb_kind {
    LMMSE_COMB_3W = 0,
    LMMSE_COMB_12W = 1,
    /* interpolated-LS baselines (no filters): */
    LMMSE_COMB_LS_HOLD = 2,     /* each subcarrier takes the LS of the latest
                                   tone at or below it (the first below it) */
    LMMSE_COMB_LS_LINEAR = 3,   /* linear between the two tones around it; the
                                   nearest tone outside the first..last tone */
    LMMSE_COMB_LS_LINEAR3 = 4,  /* "3-fold": linear at the 3W output positions
                                   tone + j S/3, held as in 3W */
    LMMSE_COMB_LS_QUADRATIC = 5,/* second-order polynomial: between tones i and
                                   i+1 the quadratic through tones i-1, i, i+1
                                   (0, 1, 2 in the first interval); the nearest
                                   tone outside the first..last tone */
    LMMSE_COMB_LS_SPLINE = 6    /* natural cubic spline through the UE's tones
                                   (zero second derivative at the first and
                                   last tone); the nearest tone outside them */
} lmmse_comb_kind;

typedef struct lmmse_comb_desc {
    int M;           /* BS antennas                                   (>= 1) */
    int K;           /* active UEs = comb offsets 0..K-1           (1..comb) */
    int comb;        /* comb spacing S: N % S == 0; 3W: S % 3 == 0;
                        12W: S <= 16                                         */
    int N;           /* used subcarriers; N / S <= 4096 and >= win (3W 3,
                        12W 12, QUADRATIC and SPLINE 3, other LS kinds 2)   */
    int N_fft;       /* FFT size (>= N)                                      */
    int kind;        /* lmmse_comb_kind                                      */
    int rsource;     /* LMMSE_R_UNIFORM or LMMSE_R_EXPONENTIAL (the filter
                        kinds; checked for every kind)                       */
    int taps;        /* EXPONENTIAL: integer taps (1..N_fft)                 */
    double tau_rms;  /* EXPONENTIAL: profile decay (> 0)                     */
    double L;        /* UNIFORM: assumed channel length in samples (> 0)     */
    double sigma2;   /* noise variance per resource element (> 0)            */
    int max_slots;   /* largest batch any call will pass (>= 1)              */
} lmmse_comb_desc;

typedef struct lmmse_comb *lmmse_comb_t;

/* Host-only check of a descriptor: OK, INVALID_ARG or UNSUPPORTED. */
int lmmse_comb_validate(const lmmse_comb_desc *desc);

/* Validates, allocates the plan's filters on the current device and designs
 * them (synchronously).  Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, HIP,
 * NOT_PD. */
int lmmse_comb_create(const lmmse_comb_desc *desc, lmmse_comb_t *out);

/* Frees the plan (synchronises the device first). */
int lmmse_comb_destroy(lmmse_comb_t comb);

/* Copies the FP64 filter classes to device complex128
 * [K][win][nout][win] (class c = b - wst_b; nout = 3 for 3W, S for 12W;
 * rows of 3W outputs past N are still designed).  Asynchronous. */
int lmmse_comb_get_filters(lmmse_comb_t comb, void *w_out, void *stream);

/* y: complex64 [slots][M][N] pilot symbol; pilots: complex64 [N], the pilot
 * on each subcarrier (nonzero); h_hat: complex64 [slots][M][K][N].  One
 * launch on `stream`. */
int lmmse_comb_estimate(lmmse_comb_t comb, int slots, const void *y,
                        const void *pilots, void *h_hat, void *stream);

/* ---- MMSE MIMO detection (Sec. IV-A, eq. 20-22; Sec. IV-C) -------------- */

/* Per (slot s, data subcarrier n), with H = h_hat[s][:][:][n] (M x K) and
 * Y = y_data[s][:][:][n] (M x T), writes X = x_out[s][:][:][n] (T x K as
 * [T][K]) solving (H^H H + sigma2 I) X^T = H^H Y (eq. 22) by Cholesky in
 * FP32, the paper's single-precision route.  h_hat: complex64
 * [slots][M][K][N] (the estimator's layout); y_data: complex64
 * [slots][M][T][N]; x_out: complex64 [slots][T][K][N]; sigma2 > 0 is the
 * noise variance per resource element with unit-power symbols.  K <= 16 and
 * T <= 16 (else UNSUPPORTED).  One launch on `stream`; a non-positive pivot
 * yields NaN symbols for that subcarrier. */
int lmmse_mmse_detect(int slots, int M, int K, int T, int N, const void *h_hat,
                      const void *y_data, double sigma2, void *x_out,
                      void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LMMSE_H */
