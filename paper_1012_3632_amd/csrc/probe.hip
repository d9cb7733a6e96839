// Access-pattern calibration: the memory traffic of a step kernel without
// its arithmetic.  One thread per site reads q population planes (element
// site of each plane, plane stride V) and writes them back, either in place
// or to a second buffer, scaled by 1.  The rate it reaches is the ceiling a
// step kernel with the same plane layout can approach when it is bound by
// HBM.  a and b may be the same buffer (no restrict qualifiers).
#include <hip/hip_runtime.h>

#include "../../include/flb.h"
#include "internal.h"

namespace flb {
namespace {

template <int Q>
__global__ __launch_bounds__(256) void k_plane_stream(const float* a,
                                                      float* b, uint32_t V) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= V) return;
    float v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = a[(size_t)i * V + s];
#pragma unroll
    for (int i = 0; i < Q; ++i) b[(size_t)i * V + s] = v[i] * 1.0f;
}

}  // namespace
}  // namespace flb

extern "C" flb_status flb_plane_stream_probe(const void* a, void* b, int32_t q, uint64_t V,
                                             int32_t repeats, void* stream) {
    if (!a || !b || (q != 9 && q != 19) || V == 0 || V >= (1ull << 31) || repeats < 1) {
        flb::set_last_error("flb_plane_stream_probe: a, b non-NULL, q 9 or 19, 0 < V < 2^31, "
                            "repeats >= 1");
        return FLB_ERR_INVALID_ARG;
    }
    const hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)((V + 255) / 256)), block(256);
    for (int r = 0; r < repeats; ++r) {
        if (q == 19)
            hipLaunchKernelGGL(flb::k_plane_stream<19>, grid, block, 0, st, (const float*)a,
                               (float*)b, (uint32_t)V);
        else
            hipLaunchKernelGGL(flb::k_plane_stream<9>, grid, block, 0, st, (const float*)a,
                               (float*)b, (uint32_t)V);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        flb::set_last_error(hipGetErrorString(e));
        return FLB_ERR_HIP;
    }
    return FLB_OK;
}
