// Launchers of paths that are not available in this build: they report
// hipErrorNotSupported, which the C ABI turns into LMMSE_ERR_HIP.
#include "internal.h"

namespace lmmse {

hipError_t launch_backward_sample(Plan&, int, const float2*, const float2*, float2*, double, bool,
                                  void*, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace lmmse
