// Instantiations and launcher of the 2-D F64 step kernels on the D2Q37 lattice
// (ping-pong and in-place even/odd).
#include <hip/hip_runtime.h>

#include "step_impl.hpp"

namespace lbmx {

hipError_t launch_step_37_f64(const int tile[3], const StepArgs &a, hipStream_t s) {
    bool done = false;
    switch (a.scheme) {
        case kSchemePingPong: done = launch_37<double, kSchemePingPong>(tile, a, s); break;
        case kSchemeInPlaceEven: done = launch_37<double, kSchemeInPlaceEven>(tile, a, s); break;
        case kSchemeInPlaceOdd: done = launch_37<double, kSchemeInPlaceOdd>(tile, a, s); break;
        default: return hipErrorInvalidValue;
    }
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}
}  // namespace lbmx
