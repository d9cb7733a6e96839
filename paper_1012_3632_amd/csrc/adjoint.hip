// Adjoint (reverse-mode) kernels of the fluctuating LB step.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace flb {

size_t adjoint_work_bytes(const StepSpec&) { return 0; }
uint32_t adjoint_slots(const StepSpec&) { return 1; }
hipError_t launch_adjoint_seed(const StepSpec&, const void*, void*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_adjoint_step(const StepSpec&, const void*, const void*, const void*, void*,
                               void*, unsigned long long, double*, uint32_t*, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace flb
