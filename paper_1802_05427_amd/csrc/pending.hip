// Launchers of paths that are not available in this build: they report
// hipErrorNotSupported, which the C ABI turns into LMMSE_ERR_HIP.
#include "internal.h"

namespace lmmse {

hipError_t launch_apply_split(const Plan&, int, const float2*, const float2*, bool, float2*,
                              hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_covariance(const Plan&, int, const float2*, double2*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_batched_filters(const Plan&, int, double2*, double2*, const double2*, double,
                                  double2*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_sample_estimate(const Plan&, int, const float2*, double, float2*, void*,
                                  hipStream_t) {
    return hipErrorNotSupported;
}
size_t sample_workspace_bytes(const lmmse_plan_desc&, int) { return 0; }
size_t backward_workspace_bytes(const lmmse_plan_desc&, int) { return 0; }
hipError_t launch_backward_fixed(Plan&, int, const float2*, const float2*, float2*, bool, void*,
                                 hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_backward_sample(Plan&, int, const float2*, const float2*, float2*, double, bool,
                                  void*, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace lmmse
