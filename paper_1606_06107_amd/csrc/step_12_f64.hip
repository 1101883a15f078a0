// Instantiations and launcher of the 1-D/2-D F64 ping-pong step kernels.
#include <hip/hip_runtime.h>

#include "step_impl.hpp"

namespace lbmx {

hipError_t launch_step_12_f64(int dim, const int tile[3], const StepArgs &a, hipStream_t s) {
    bool done = false;
    switch (a.scheme) {
        case kSchemePingPong: done = launch_12<double, kSchemePingPong>(dim, tile, a, s); break;
        default: return launch_step_12_f64_inplace(dim, tile, a, s);
    }
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}
}  // namespace lbmx
