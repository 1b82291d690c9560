// Host side of the C ABI declared in include/lmmse.h: argument checks, the
// block plan, plan-owned device memory and dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

using namespace lmmse;

// The opaque handle of the C ABI is the plan itself.
struct lmmse_plan : lmmse::Plan {};

namespace {

constexpr int kMaxK = 64;
constexpr int kMaxWindow = 1344;     // fixed design: 3 Wn complex doubles of LDS (<= 64 KB)
constexpr int kRTs[] = {1, 2, 4, 8, 9, 13, 15, 17};

#define LMMSE_HIP_TRY(expr)                       \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) return LMMSE_ERR_HIP; \
    } while (0)

int block_plan_impl(int N, int B, int Wn, std::vector<int>& starts, std::vector<int>& offs,
                    std::vector<int>& cls, std::vector<int>& class_off) {
    if (N <= 0 || B <= 0 || Wn <= 0) return LMMSE_ERR_INVALID_ARG;
    if (N % B != 0 || Wn < B || Wn > N || ((Wn - B) & 1)) return LMMSE_ERR_UNSUPPORTED;
    const int nb = N / B, halo = (Wn - B) / 2;
    starts.assign(nb, 0);
    offs.assign(nb, 0);
    cls.assign(nb, 0);
    class_off.clear();
    for (int b = 0; b < nb; ++b) {
        const int s = std::min(std::max(b * B - halo, 0), N - Wn);
        starts[b] = s;
        offs[b] = b * B - s;
        auto it = std::find(class_off.begin(), class_off.end(), offs[b]);
        if (it == class_off.end()) {
            cls[b] = (int)class_off.size();
            class_off.push_back(offs[b]);
        } else {
            cls[b] = (int)(it - class_off.begin());
        }
    }
    return LMMSE_OK;
}

int validate(const lmmse_plan_desc* d) {
    if (!d) return LMMSE_ERR_INVALID_ARG;
    if (d->M < 1 || d->K < 1 || d->N < 1 || d->N_fft < d->N || d->B < 1 || d->Wn < 1 ||
        d->max_slots < 1)
        return LMMSE_ERR_INVALID_ARG;
    if (d->rsource < LMMSE_R_UNIFORM || d->rsource > LMMSE_R_USER_R) return LMMSE_ERR_INVALID_ARG;
    if (d->precision < LMMSE_FP32 || d->precision > LMMSE_FP16X3) return LMMSE_ERR_INVALID_ARG;
    if (d->rsource == LMMSE_R_EXPONENTIAL &&
        (d->taps < 1 || d->taps > d->N_fft || !(d->tau_rms > 0.0) || !std::isfinite(d->tau_rms)))
        return LMMSE_ERR_INVALID_ARG;
    if (d->rsource == LMMSE_R_UNIFORM && (!(d->L > 0.0) || !std::isfinite(d->L)))
        return LMMSE_ERR_INVALID_ARG;
    if ((d->rsource == LMMSE_R_UNIFORM || d->rsource == LMMSE_R_EXPONENTIAL ||
         d->rsource == LMMSE_R_USER_R) &&
        (!(d->sigma2 > 0.0) || !std::isfinite(d->sigma2)))
        return LMMSE_ERR_INVALID_ARG;
    if (d->K > kMaxK) return LMMSE_ERR_UNSUPPORTED;
    if (d->N % d->B != 0 || d->Wn < d->B || d->Wn > d->N || ((d->Wn - d->B) & 1))
        return LMMSE_ERR_UNSUPPORTED;
    if (d->Wn > kMaxWindow) return LMMSE_ERR_UNSUPPORTED;
    const long long cols = (long long)d->max_slots * d->M * d->K;
    // per-coefficient kernels run one work-item per coefficient, and a grid's
    // work-items stay below 2^32
    if (cols * d->N >= (1LL << 32)) return LMMSE_ERR_UNSUPPORTED;
    // windows wider than the workspace-resident design: the push-through form
    // (M x M systems), FP32 product only
    if (d->rsource == LMMSE_R_SAMPLE && d->Wn > kMaxSampleWindowLarge &&
        (d->M > kMaxPushthroughAntennas || d->precision != LMMSE_FP32))
        return LMMSE_ERR_UNSUPPORTED;
    return LMMSE_OK;
}

// Row tiles per workgroup: padded tiles, charged 5% per row group (each
// group re-reads the window's inputs and redoes their staging).
void choose_row_tiles(int B, int max_rt, int& RT, int& rgroups) {
    const int T = (2 * B + 15) / 16;
    double best = -1.0;
    for (int rt : kRTs) {
        if (rt > max_rt) continue;
        const int g = (T + rt - 1) / rt;
        const double cost = (double)g * rt * (1.0 + 0.05 * g);
        if (best < 0.0 || cost < best) {
            best = cost;
            RT = rt;
            rgroups = g;
        }
    }
}

bool fixed_source(int rs) { return rs == LMMSE_R_UNIFORM || rs == LMMSE_R_EXPONENTIAL; }
// sources whose filters the plan designs from a correlation it holds
bool designed_source(int rs) { return fixed_source(rs) || rs == LMMSE_R_USER_R; }

template <typename T>
int dev_alloc(T*& p, size_t count) {
    p = nullptr;
    if (count == 0) return LMMSE_OK;
    if (hipMalloc((void**)&p, count * sizeof(T)) != hipSuccess) {
        p = nullptr;
        return LMMSE_ERR_HIP;
    }
    return LMMSE_OK;
}

void free_plan(lmmse_plan* p) {
    if (!p) return;
    void* ptrs[] = {p->d_starts, p->d_classes, p->d_offsets, p->d_bstarts, p->d_class_off, p->w64,
                    p->ainv,     p->rwin,      p->dwork,     p->rd,        p->wf32,      p->whi,
                    p->wlo,      p->twiddle,   p->status,    p->dscal};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->join) (void)hipEventDestroy(p->join);
    if (p->side) (void)hipStreamDestroy(p->side);
    delete p;
}

int check_device() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return LMMSE_ERR_NO_DEVICE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LMMSE_ERR_NO_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return LMMSE_ERR_NO_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LMMSE_ERR_NO_DEVICE;
    return LMMSE_OK;
}

}  // namespace

namespace lmmse {

// H_LS staging in the workspace, rounded up to 256 bytes so that what follows
// it (the sample path's filters) stays 16-byte aligned for the LDS copies.
size_t hls_bytes(const lmmse_plan_desc& d, int slots) {
    return ((size_t)slots * d.M * d.K * d.N * sizeof(float2) + 255) & ~(size_t)255;
}

size_t forward_workspace_bytes(const lmmse_plan_desc& d, int slots) {
    if (slots <= 0) return 0;
    if (d.rsource == LMMSE_R_SAMPLE) return sample_workspace_bytes(d, slots);
    Plan tmp;
    tmp.d = d;
    return apply_fusable(tmp) ? 0 : hls_bytes(d, slots);
}

int plan_device(lmmse_plan_t plan) { return plan->device; }

size_t fixed_bank_f32_elems(const Plan& p) { return (size_t)p.n_classes * 2 * p.G16 * p.Rpad * 4; }
size_t split_bank_elems(const Plan& p) { return (size_t)p.n_classes * p.G16 * p.Rpad * 32; }

}  // namespace lmmse

extern "C" {

const char* lmmse_status_string(int s) {
    switch (s) {
        case LMMSE_OK: return "ok";
        case LMMSE_ERR_INVALID_ARG: return "invalid argument";
        case LMMSE_ERR_UNSUPPORTED: return "unsupported plan shape";
        case LMMSE_ERR_WORKSPACE: return "workspace missing or too small";
        case LMMSE_ERR_HIP: return "HIP runtime error";
        case LMMSE_ERR_NOT_PD: return "matrix not positive definite";
        case LMMSE_ERR_NOT_READY: return "filters not designed or set";
        case LMMSE_ERR_NO_DEVICE: return "no gfx950 device";
        case LMMSE_ERR_RANGE: return "value outside the FP16 split range";
        default: return "unknown status";
    }
}

int lmmse_version(void) { return 10100; }

int lmmse_plan_validate(const lmmse_plan_desc* desc) { return validate(desc); }

int lmmse_block_plan(int N, int B, int Wn, int* starts, int* offsets, int* classes, int* n_classes) {
    std::vector<int> s, o, c, co;
    const int rc = block_plan_impl(N, B, Wn, s, o, c, co);
    if (rc != LMMSE_OK) return rc;
    for (size_t b = 0; b < s.size(); ++b) {
        if (starts) starts[b] = s[b];
        if (offsets) offsets[b] = o[b];
        if (classes) classes[b] = c[b];
    }
    if (n_classes) *n_classes = (int)co.size();
    return LMMSE_OK;
}

int lmmse_workspace_size(const lmmse_plan_desc* desc, int slots, size_t* bytes) {
    const int v = validate(desc);
    if (v != LMMSE_OK) return v;
    if (!bytes || slots < 0 || slots > desc->max_slots) return LMMSE_ERR_INVALID_ARG;
    const size_t need =
        std::max(forward_workspace_bytes(*desc, slots), backward_workspace_bytes(*desc, slots));
    *bytes = need;
    return LMMSE_OK;
}

int lmmse_plan_create(const lmmse_plan_desc* desc, lmmse_plan_t* out) {
    if (!out) return LMMSE_ERR_INVALID_ARG;
    const int v = validate(desc);
    if (v != LMMSE_OK) return v;
    const int dv = check_device();
    if (dv != LMMSE_OK) return dv;

    lmmse_plan* p = new (std::nothrow) lmmse_plan();
    if (!p) return LMMSE_ERR_HIP;
    p->d = *desc;
    (void)hipGetDevice(&p->device);
    std::vector<int> offs;
    block_plan_impl(desc->N, desc->B, desc->Wn, p->h_starts, p->h_offsets, p->h_classes,
                    p->h_class_off);
    p->nb = desc->N / desc->B;
    p->halo = (desc->Wn - desc->B) / 2;
    if (desc->rsource == LMMSE_R_USER_R) {
        // a caller correlation need not be Toeplitz: one filter per block
        p->h_class_off = p->h_offsets;
        for (int b = 0; b < p->nb; ++b) p->h_classes[b] = b;
    }
    p->n_classes = (int)p->h_class_off.size();
    // split-precision kernels double-buffer three filter parts in LDS: RT <= 13
    choose_row_tiles(desc->B, desc->precision == LMMSE_FP32 ? 17 : 13, p->RT, p->rgroups);
    // the sample path's split kernel holds one window's filter parts compactly
    // (two buffers of 8 RT rows x 4 slots per part): 17 tiles fit, so a block
    // of up to 136 outputs reads its window once
    choose_row_tiles(desc->B, 17, p->sRT, p->srgroups);
    p->Rpad = p->RT * 16 * p->rgroups;
    p->G8 = (desc->Wn + 7) / 8;
    p->G16 = (desc->Wn + 15) / 16;
    p->lo_scale = desc->precision == LMMSE_FP16X3 ? 2048.0f : 1.0f;
    p->design_tau = desc->tau_rms;
    p->design_sigma2 = desc->sigma2;

    const int Wn = desc->Wn, K = desc->K;
    const bool has_bank = desc->rsource != LMMSE_R_SAMPLE;
    int rc = LMMSE_OK;
    auto fail = [&](int code) {
        free_plan(p);
        return code;
    };
    if ((rc = dev_alloc(p->d_starts, p->nb)) || (rc = dev_alloc(p->d_classes, p->nb)) ||
        (rc = dev_alloc(p->d_offsets, p->nb)) || (rc = dev_alloc(p->d_bstarts, p->nb)) ||
        (rc = dev_alloc(p->d_class_off, p->n_classes)) || (rc = dev_alloc(p->twiddle, K)) ||
        (rc = dev_alloc(p->status, 2)) || (rc = dev_alloc(p->dscal, 4)) ||
        (rc = dev_alloc(p->rd, 3 * (size_t)Wn)))
        return fail(rc);
    if (has_bank) {
        const size_t ainv_mats = desc->rsource == LMMSE_R_USER_R ? (size_t)p->nb : 1;
        if ((rc = dev_alloc(p->w64, (size_t)p->n_classes * desc->B * Wn)) ||
            (rc = dev_alloc(p->ainv, ainv_mats * Wn * Wn)) ||
            (rc = dev_alloc(p->wf32, fixed_bank_f32_elems(*p))))
            return fail(rc);
        if (desc->precision != LMMSE_FP32 &&
            ((rc = dev_alloc(p->whi, split_bank_elems(*p))) ||
             (rc = dev_alloc(p->wlo, split_bank_elems(*p)))))
            return fail(rc);
    }
    if (desc->rsource == LMMSE_R_USER_R &&
        ((rc = dev_alloc(p->rwin, (size_t)p->nb * Wn * Wn)) ||
         (rc = dev_alloc(p->dwork, user_corr_scratch_bytes(*desc) / sizeof(double2)))))
        return fail(rc);
    std::vector<float2> tw(K);
    for (int r = 0; r < K; ++r) {
        const double a = 2.0 * M_PI * r / K;
        tw[r] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    int zero[2] = {0, 0};
    std::vector<int> bstarts(p->nb);
    for (int b = 0; b < p->nb; ++b) bstarts[b] = b * desc->B;
    if (hipMemcpy(p->d_starts, p->h_starts.data(), p->nb * sizeof(int), hipMemcpyHostToDevice) ||
        hipMemcpy(p->d_bstarts, bstarts.data(), p->nb * sizeof(int), hipMemcpyHostToDevice) ||
        hipMemcpy(p->d_classes, p->h_classes.data(), p->nb * sizeof(int), hipMemcpyHostToDevice) ||
        hipMemcpy(p->d_offsets, p->h_offsets.data(), p->nb * sizeof(int), hipMemcpyHostToDevice) ||
        hipMemcpy(p->d_class_off, p->h_class_off.data(), p->n_classes * sizeof(int),
                  hipMemcpyHostToDevice) ||
        hipMemcpy(p->twiddle, tw.data(), K * sizeof(float2), hipMemcpyHostToDevice) ||
        hipMemcpy(p->status, zero, sizeof(zero), hipMemcpyHostToDevice))
        return fail(LMMSE_ERR_HIP);
    if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->join, hipEventDisableTiming) != hipSuccess)
        return fail(LMMSE_ERR_HIP);
    if (has_bank) {
        const size_t bytes = fixed_bank_f32_elems(*p) * sizeof(float4);
        if (hipMemset(p->wf32, 0, bytes) != hipSuccess) return fail(LMMSE_ERR_HIP);
    }
    // r_d is not used by a caller correlation: zero, so that the design
    // backward's r_d terms vanish
    if (hipMemset(p->rd, 0, 3 * (size_t)Wn * sizeof(double2)) != hipSuccess) return fail(LMMSE_ERR_HIP);
    if (fixed_source(desc->rsource)) {
        if (launch_fixed_design(*p, desc->tau_rms, desc->sigma2, 0) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)
            return fail(LMMSE_ERR_HIP);
        int st[2];
        if (hipMemcpy(st, p->status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(LMMSE_ERR_HIP);
        if (st[0] != 0) return fail(st[0]);
        p->ready = true;
    }
    *out = p;
    return LMMSE_OK;
}

int lmmse_plan_destroy(lmmse_plan_t plan) {
    if (!plan) return LMMSE_ERR_INVALID_ARG;
    (void)hipDeviceSynchronize();
    free_plan(plan);
    return LMMSE_OK;
}

int lmmse_plan_get_desc(lmmse_plan_t plan, lmmse_plan_desc* out) {
    if (!plan || !out) return LMMSE_ERR_INVALID_ARG;
    *out = plan->d;
    out->tau_rms = plan->design_tau;
    out->sigma2 = plan->design_sigma2;
    return LMMSE_OK;
}

int lmmse_set_design(lmmse_plan_t plan, double tau_rms, double sigma2, void* stream) {
    if (!plan) return LMMSE_ERR_INVALID_ARG;
    if (plan->d.rsource == LMMSE_R_SAMPLE) {
        // only the noise variance: the filters come from each batch's data
        if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return LMMSE_ERR_INVALID_ARG;
        plan->design_sigma2 = sigma2;
        return LMMSE_OK;
    }
    if (plan->d.rsource == LMMSE_R_USER_R) {
        // only the noise variance; redesigned from the caller's correlation
        // once one has been set
        if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return LMMSE_ERR_INVALID_ARG;
        plan->design_sigma2 = sigma2;
        if (plan->have_corr) {
            LMMSE_HIP_TRY(launch_user_corr_design(*plan, sigma2, (hipStream_t)stream));
            plan->ready = true;
        }
        return LMMSE_OK;
    }
    if (!fixed_source(plan->d.rsource)) return LMMSE_ERR_UNSUPPORTED;
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return LMMSE_ERR_INVALID_ARG;
    if (plan->d.rsource == LMMSE_R_EXPONENTIAL && (!(tau_rms > 0.0) || !std::isfinite(tau_rms)))
        return LMMSE_ERR_INVALID_ARG;
    const double tau = plan->d.rsource == LMMSE_R_EXPONENTIAL ? tau_rms : plan->design_tau;
    LMMSE_HIP_TRY(launch_fixed_design(*plan, tau, sigma2, (hipStream_t)stream));
    plan->design_tau = tau;
    plan->design_sigma2 = sigma2;
    plan->ready = true;
    return LMMSE_OK;
}

int lmmse_set_filters(lmmse_plan_t plan, const void* w, void* stream) {
    if (!plan || !w) return LMMSE_ERR_INVALID_ARG;
    if (plan->d.rsource != LMMSE_R_USER) return LMMSE_ERR_UNSUPPORTED;
    const size_t bytes = (size_t)plan->n_classes * plan->d.B * plan->d.Wn * sizeof(double2);
    LMMSE_HIP_TRY(hipMemcpyAsync(plan->w64, w, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    LMMSE_HIP_TRY(launch_pack_banks(*plan, (hipStream_t)stream));
    plan->ready = true;
    return LMMSE_OK;
}

int lmmse_set_input_scale(lmmse_plan_t plan, double scale) {
    if (!plan) return LMMSE_ERR_INVALID_ARG;
    int e = 0;
    if (!(scale > 0.0) || !std::isfinite(scale) || std::frexp(scale, &e) != 0.5 || e < -59 || e > 61)
        return LMMSE_ERR_INVALID_ARG;
    plan->in_scale = (float)scale;
    return LMMSE_OK;
}

int lmmse_set_correlation(lmmse_plan_t plan, const void* r, void* stream) {
    if (!plan || !r) return LMMSE_ERR_INVALID_ARG;
    if (plan->d.rsource != LMMSE_R_USER_R) return LMMSE_ERR_UNSUPPORTED;
    LMMSE_HIP_TRY(launch_user_corr_gather(*plan, (const double2*)r, (hipStream_t)stream));
    LMMSE_HIP_TRY(launch_user_corr_design(*plan, plan->design_sigma2, (hipStream_t)stream));
    plan->have_corr = true;
    plan->ready = true;
    return LMMSE_OK;
}

int lmmse_get_filters(lmmse_plan_t plan, void* w_out, void* stream) {
    if (!plan || !w_out) return LMMSE_ERR_INVALID_ARG;
    if (plan->d.rsource == LMMSE_R_SAMPLE) return LMMSE_ERR_UNSUPPORTED;
    if (!plan->ready) return LMMSE_ERR_NOT_READY;
    const size_t bytes = (size_t)plan->n_classes * plan->d.B * plan->d.Wn * sizeof(double2);
    LMMSE_HIP_TRY(hipMemcpyAsync(w_out, plan->w64, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return LMMSE_OK;
}

int lmmse_despread(lmmse_plan_t plan, int slots, const void* y, const void* pilots, void* h_ls,
                   void* stream) {
    if (!plan || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (slots == 0) return LMMSE_OK;
    if (!y || !pilots || !h_ls) return LMMSE_ERR_INVALID_ARG;
    LMMSE_HIP_TRY(launch_despread(*plan, slots, (const float2*)y, (const float2*)pilots,
                                  (float2*)h_ls, (hipStream_t)stream));
    return LMMSE_OK;
}

static int apply_dispatch(lmmse_plan_t plan, int slots, const float2* x, const float2* pilots,
                          bool fused, float2* out, hipStream_t st) {
    if (plan->d.precision == LMMSE_FP32)
        LMMSE_HIP_TRY(launch_apply_f32(*plan, slots, x, pilots, fused, out, st));
    else
        LMMSE_HIP_TRY(launch_apply_split(*plan, slots, x, pilots, fused, out, st));
    return LMMSE_OK;
}

int lmmse_apply(lmmse_plan_t plan, int slots, const void* h_ls, void* h_hat, void* stream) {
    if (!plan || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (plan->d.rsource == LMMSE_R_SAMPLE) return LMMSE_ERR_UNSUPPORTED;
    if (!plan->ready) return LMMSE_ERR_NOT_READY;
    if (slots == 0) return LMMSE_OK;
    if (!h_ls || !h_hat) return LMMSE_ERR_INVALID_ARG;
    return apply_dispatch(plan, slots, (const float2*)h_ls, nullptr, false, (float2*)h_hat,
                          (hipStream_t)stream);
}

int lmmse_covariance(lmmse_plan_t plan, int slots, const void* h_ls, void* r_win, void* stream) {
    if (!plan || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (slots == 0) return LMMSE_OK;
    if (!h_ls || !r_win) return LMMSE_ERR_INVALID_ARG;
    LMMSE_HIP_TRY(launch_covariance(*plan, slots, (const float2*)h_ls, (double2*)r_win,
                                    (hipStream_t)stream));
    return LMMSE_OK;
}

int lmmse_sample_filters_workspace_size(const lmmse_plan_desc* desc, int slots, size_t* bytes) {
    const int v = validate(desc);
    if (v != LMMSE_OK) return v;
    if (!bytes || slots < 0 || slots > desc->max_slots) return LMMSE_ERR_INVALID_ARG;
    const long long nmat = (long long)slots * desc->K * (desc->N / desc->B);
    *bytes = desc->Wn <= kMaxSampleWindowReg
                 ? 0
                 : (size_t)nmat * desc->Wn * desc->Wn * sizeof(double2) +
                       sweep_scratch_bytes(desc->Wn, nmat);
    return LMMSE_OK;
}

int lmmse_sample_filters(lmmse_plan_t plan, int slots, const void* r_win, double sigma2,
                         void* w_out, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (!(sigma2 >= 0.0) || !std::isfinite(sigma2)) return LMMSE_ERR_INVALID_ARG;
    if (slots == 0) return LMMSE_OK;
    if (!r_win || !w_out) return LMMSE_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    const long long nmat = (long long)slots * plan->d.K * plan->nb;
    const double lam = sigma2 / plan->d.K;
    if (plan->d.Wn <= kMaxSampleWindowReg) {
        LMMSE_HIP_TRY(launch_batched_filters(*plan, nmat, (const double2*)r_win, lam, (double2*)w_out,
                                             nullptr, st));
        return LMMSE_OK;
    }
    // wider windows: the sweep inverse of a copy of the windows in ws
    size_t need = 0;
    lmmse_sample_filters_workspace_size(&plan->d, slots, &need);
    if (!ws || ws_bytes < need) return LMMSE_ERR_WORKSPACE;
    const int Wn = plan->d.Wn;
    double2* amat = (double2*)ws;
    double2* scratch = amat + nmat * Wn * Wn;
    LMMSE_HIP_TRY(hipMemcpyAsync(amat, r_win, (size_t)nmat * Wn * Wn * sizeof(double2),
                                 hipMemcpyDeviceToDevice, st));
    LMMSE_HIP_TRY(launch_sweep_inverse(nmat, 0, Wn, plan->d.K, plan->nb, lam, amat, scratch,
                                       plan->status, st));
    LMMSE_HIP_TRY(launch_large_filters(nmat, amat, plan->d_offsets, plan->d.B, Wn, plan->nb, lam,
                                       (double2*)w_out, false, st));
    return LMMSE_OK;
}

int lmmse_estimate(lmmse_plan_t plan, int slots, const void* y, const void* pilots, double sigma2,
                   void* h_hat, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return LMMSE_ERR_INVALID_ARG;
    if (slots == 0) return LMMSE_OK;
    if (!y || !pilots || !h_hat) return LMMSE_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    if (plan->d.rsource == LMMSE_R_SAMPLE) {
        if (!ws || ws_bytes < sample_workspace_bytes(plan->d, slots)) return LMMSE_ERR_WORKSPACE;
        plan->design_sigma2 = sigma2;   // the backward of this estimate uses it
        float2* hls = (float2*)ws;
        LMMSE_HIP_TRY(launch_despread(*plan, slots, (const float2*)y, (const float2*)pilots, hls, st));
        LMMSE_HIP_TRY(launch_sample_estimate(*plan, slots, hls, sigma2 / plan->d.K, (float2*)h_hat,
                                             (char*)ws + hls_bytes(plan->d, slots), st));
        return LMMSE_OK;
    }
    if (designed_source(plan->d.rsource) && sigma2 != plan->design_sigma2) {
        const int rc = lmmse_set_design(plan, plan->design_tau, sigma2, stream);
        if (rc != LMMSE_OK) return rc;
    }
    if (!plan->ready) return LMMSE_ERR_NOT_READY;
    if (apply_fusable(*plan))
        return apply_dispatch(plan, slots, (const float2*)y, (const float2*)pilots, true,
                              (float2*)h_hat, st);
    if (!ws || ws_bytes < hls_bytes(plan->d, slots)) return LMMSE_ERR_WORKSPACE;
    LMMSE_HIP_TRY(launch_despread(*plan, slots, (const float2*)y, (const float2*)pilots, (float2*)ws, st));
    return apply_dispatch(plan, slots, (const float2*)ws, nullptr, false, (float2*)h_hat, st);
}

int lmmse_estimate_ls(lmmse_plan_t plan, int slots, const void* h_ls, double sigma2, void* h_hat,
                      void* ws, size_t ws_bytes, void* stream) {
    if (!plan || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return LMMSE_ERR_INVALID_ARG;
    if (slots == 0) return LMMSE_OK;
    if (!h_ls || !h_hat) return LMMSE_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    if (plan->d.rsource == LMMSE_R_SAMPLE) {
        // same workspace layout as lmmse_estimate; its LS area stays unused
        if (!ws || ws_bytes < sample_workspace_bytes(plan->d, slots)) return LMMSE_ERR_WORKSPACE;
        plan->design_sigma2 = sigma2;
        LMMSE_HIP_TRY(launch_sample_estimate(*plan, slots, (const float2*)h_ls, sigma2 / plan->d.K,
                                             (float2*)h_hat, (char*)ws + hls_bytes(plan->d, slots),
                                             st));
        return LMMSE_OK;
    }
    if (designed_source(plan->d.rsource) && sigma2 != plan->design_sigma2) {
        const int rc = lmmse_set_design(plan, plan->design_tau, sigma2, stream);
        if (rc != LMMSE_OK) return rc;
    }
    if (!plan->ready) return LMMSE_ERR_NOT_READY;
    return apply_dispatch(plan, slots, (const float2*)h_ls, nullptr, false, (float2*)h_hat, st);
}

// The design a sample forward keeps for its backward: W rows [nmat][B][Wn],
// then A^-1 [nmat][Wn][Wn], FP64 complex; windows the resident design holds.
static size_t kept_design_bytes(const lmmse_plan_desc& d, int slots) {
    if (d.rsource != LMMSE_R_SAMPLE || !resident_design_fits(d.Wn) || slots <= 0) return 0;
    const long long nmat = (long long)slots * d.K * (d.N / d.B);
    return (size_t)nmat * ((size_t)d.B * d.Wn + (size_t)d.Wn * d.Wn) * sizeof(double2);
}

int lmmse_design_state_size(lmmse_plan_t plan, int slots, size_t* bytes) {
    if (!plan || !bytes || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    *bytes = kept_design_bytes(plan->d, slots);
    return LMMSE_OK;
}

int lmmse_estimate_ls_keep(lmmse_plan_t plan, int slots, const void* h_ls, double sigma2, void* h_hat,
                           void* state, size_t state_bytes, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return LMMSE_ERR_INVALID_ARG;
    if (plan->d.rsource != LMMSE_R_SAMPLE || !resident_design_fits(plan->d.Wn))
        return LMMSE_ERR_UNSUPPORTED;
    if (slots == 0) return LMMSE_OK;
    if (!h_ls || !h_hat || !state) return LMMSE_ERR_INVALID_ARG;
    if (state_bytes < kept_design_bytes(plan->d, slots)) return LMMSE_ERR_WORKSPACE;
    if (!ws || ws_bytes < sample_workspace_bytes(plan->d, slots)) return LMMSE_ERR_WORKSPACE;
    plan->design_sigma2 = sigma2;
    const long long nmat = (long long)slots * plan->d.K * plan->nb;
    double2* kw = (double2*)state;
    double2* ka = kw + nmat * plan->d.B * plan->d.Wn;
    LMMSE_HIP_TRY(launch_sample_estimate(*plan, slots, (const float2*)h_ls, sigma2 / plan->d.K,
                                         (float2*)h_hat, (char*)ws + hls_bytes(plan->d, slots),
                                         (hipStream_t)stream, kw, ka));
    return LMMSE_OK;
}

// The backward's launches (every entry point): d_hls, and the parameter
// gradients into plan->dscal when want; kept: a sample plan's design kept by
// lmmse_estimate_ls_keep (null: designed again).
static int backward_launch(lmmse_plan_t plan, int slots, const void* h_ls, const void* g, void* d_hls,
                           bool want, void* ws, size_t ws_bytes, hipStream_t st,
                           const void* kept = nullptr) {
    if (!plan || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (slots > 0 && (!h_ls || !g || !d_hls)) return LMMSE_ERR_INVALID_ARG;
    // windows wider than 256: no gradient through the sample covariance, and
    // no design-parameter gradients of the designed filters (dX alone is
    // supported for fixed, caller-correlation and caller filters)
    if (plan->d.Wn > kMaxSampleWindowLarge &&
        (plan->d.rsource == LMMSE_R_SAMPLE || (want && plan->d.rsource != LMMSE_R_USER)))
        return LMMSE_ERR_UNSUPPORTED;
    const size_t need = backward_workspace_bytes(plan->d, slots);
    if (need && (!ws || ws_bytes < need)) return LMMSE_ERR_WORKSPACE;
    if (plan->d.rsource == LMMSE_R_SAMPLE) {
        const long long nmat = (long long)slots * plan->d.K * plan->nb;
        const double2* kw = (const double2*)kept;
        const double2* ka = kw ? kw + nmat * plan->d.B * plan->d.Wn : nullptr;
        LMMSE_HIP_TRY(launch_backward_sample(*plan, slots, (const float2*)h_ls, (const float2*)g,
                                             (float2*)d_hls, plan->design_sigma2 / plan->d.K, want,
                                             ws, st, kw, ka));
    } else {
        if (!plan->ready) return LMMSE_ERR_NOT_READY;
        LMMSE_HIP_TRY(launch_backward_fixed(*plan, slots, (const float2*)h_ls, (const float2*)g,
                                            (float2*)d_hls, want && plan->d.rsource != LMMSE_R_USER,
                                            ws, st));
    }
    return LMMSE_OK;
}

int lmmse_backward(lmmse_plan_t plan, int slots, const void* h_ls, const void* g, void* d_hls,
                   double* d_tau, double* d_sigma2, void* ws, size_t ws_bytes, void* stream) {
    const bool want = d_tau || d_sigma2;
    const hipStream_t st = (hipStream_t)stream;
    const int rc = backward_launch(plan, slots, h_ls, g, d_hls, want, ws, ws_bytes, st);
    if (rc != LMMSE_OK) return rc;
    double h[4] = {NAN, NAN, NAN, NAN};
    if (want) {
        LMMSE_HIP_TRY(hipStreamSynchronize(st));
        if (plan->d.rsource != LMMSE_R_USER)
            LMMSE_HIP_TRY(hipMemcpy(h, plan->dscal, 2 * sizeof(double), hipMemcpyDeviceToHost));
        if (d_tau) *d_tau = plan->d.rsource == LMMSE_R_EXPONENTIAL ? h[0] : NAN;
        if (d_sigma2) *d_sigma2 = plan->d.rsource == LMMSE_R_USER ? NAN : h[1] / plan->d.K;
    }
    return LMMSE_OK;
}

int lmmse_backward_dev(lmmse_plan_t plan, int slots, const void* h_ls, const void* g, void* d_hls,
                       void* d_params, void* ws, size_t ws_bytes, void* stream) {
    const hipStream_t st = (hipStream_t)stream;
    const int rc = backward_launch(plan, slots, h_ls, g, d_hls, d_params != nullptr, ws, ws_bytes, st);
    if (rc != LMMSE_OK || !d_params) return rc;
    LMMSE_HIP_TRY(launch_params_out(*plan, (double*)d_params, st));   // NaN where the host call gives NaN
    return LMMSE_OK;
}

int lmmse_backward_kept(lmmse_plan_t plan, int slots, const void* h_ls, const void* g, void* d_hls,
                        void* d_params, const void* state, size_t state_bytes, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!plan || slots < 0 || slots > plan->d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (plan->d.rsource != LMMSE_R_SAMPLE || !resident_design_fits(plan->d.Wn))
        return LMMSE_ERR_UNSUPPORTED;
    if (slots > 0 && (!state || state_bytes < kept_design_bytes(plan->d, slots)))
        return state ? LMMSE_ERR_WORKSPACE : LMMSE_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    const int rc = backward_launch(plan, slots, h_ls, g, d_hls, d_params != nullptr, ws, ws_bytes, st,
                                   state);
    if (rc != LMMSE_OK || !d_params) return rc;
    LMMSE_HIP_TRY(launch_params_out(*plan, (double*)d_params, st));
    return LMMSE_OK;
}

int lmmse_sync_status(lmmse_plan_t plan, void* stream, int* info) {
    if (!plan) return LMMSE_ERR_INVALID_ARG;
    LMMSE_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int st[2] = {0, -1};
    LMMSE_HIP_TRY(hipMemcpy(st, plan->status, sizeof(st), hipMemcpyDeviceToHost));
    if (info) *info = st[0] ? st[1] : -1;
    if (st[0]) {
        int zero[2] = {0, 0};
        LMMSE_HIP_TRY(hipMemcpy(plan->status, zero, sizeof(zero), hipMemcpyHostToDevice));
    }
    return st[0];
}

}  // extern "C"
