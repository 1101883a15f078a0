// Instantiations and launcher of the 1-D/2-D F32 ping-pong step kernels.
#include <hip/hip_runtime.h>

#include "step_impl.hpp"

namespace lbmx {

hipError_t launch_step_12_f32(int dim, const int tile[3], const StepArgs &a, hipStream_t s) {
    bool done = false;
    switch (a.scheme) {
        case kSchemePingPong: done = launch_12<float, kSchemePingPong>(dim, tile, a, s); break;
        default: return launch_step_12_f32_inplace(dim, tile, a, s);
    }
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}
}  // namespace lbmx
