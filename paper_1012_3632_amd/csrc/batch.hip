// Batched replicas (placeholder until the persistent batched kernel lands).
#include <hip/hip_runtime.h>

#include "../../include/flb.h"

extern "C" {

flb_status flb_batch_query_sizes(const flb_params*, int32_t, const int32_t*, size_t*, size_t*,
                                 size_t*) {
    return FLB_ERR_UNSUPPORTED;
}
flb_status flb_batch_init(const flb_params*, int32_t, const int32_t*, const uint64_t*, void*,
                          void*, void*, void*, void*, flb_batch**) {
    return FLB_ERR_UNSUPPORTED;
}
flb_status flb_batch_step(flb_batch*, int64_t, int32_t, void*) { return FLB_ERR_UNSUPPORTED; }
flb_status flb_batch_moments(flb_batch*, double*, double*, int64_t*, void*) {
    return FLB_ERR_UNSUPPORTED;
}
flb_status flb_batch_state(const flb_batch*, void**, void**, uint64_t*) {
    return FLB_ERR_UNSUPPORTED;
}
flb_status flb_batch_graph_capture(flb_batch*, int64_t, int32_t, void*) {
    return FLB_ERR_UNSUPPORTED;
}
flb_status flb_batch_graph_launch(flb_batch*, void*) { return FLB_ERR_UNSUPPORTED; }
flb_status flb_batch_destroy(flb_batch*) { return FLB_ERR_UNSUPPORTED; }
flb_status flb_batch_autotune(flb_batch*, int32_t, int32_t*, double*, void*) {
    return FLB_ERR_UNSUPPORTED;
}

}  // extern "C"
