// Instantiations and launcher of the 1-D/2-D F32 in-place (even/odd) step kernels.
#include <hip/hip_runtime.h>

#include "step_impl.hpp"

namespace lbmx {

hipError_t launch_step_12_f32_inplace(int dim, const int tile[3], const StepArgs &a, hipStream_t s) {
    bool done = false;
    switch (a.scheme) {
        case kSchemeInPlaceEven: done = launch_12<float, kSchemeInPlaceEven>(dim, tile, a, s); break;
        case kSchemeInPlaceOdd: done = launch_12<float, kSchemeInPlaceOdd>(dim, tile, a, s); break;
        default: return hipErrorInvalidValue;
    }
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}
}  // namespace lbmx
