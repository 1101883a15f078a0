// Instantiations and launcher of the 1-D/2-D FP32 step kernels.
#include <hip/hip_runtime.h>

#include "step_impl.hpp"

namespace lbmx {

hipError_t launch_step_12_f32(int dim, const int tile[3], const StepArgs &a, hipStream_t s) {
    const dim3 grid(a.ntiles);
    bool done = false;
#define L1(TXv, TYv)                                                                  \
    if (!done && dim == 1 && tile[0] == TXv) {                                        \
        hipLaunchKernelGGL((k_step_12<float, 1, TXv, 1>), grid, dim3(TXv), 0, s, a);     \
        done = true;                                                                  \
    }
#define L2(TXv, TYv)                                                                  \
    if (!done && dim == 2 && tile[0] == TXv && tile[1] == TYv) {                      \
        hipLaunchKernelGGL((k_step_12<float, 2, TXv, TYv>), grid, dim3(TXv * TYv), 0, s, a); \
        done = true;                                                                  \
    }
    LBMX_TILES_1D(L1)
    LBMX_TILES_2D(L2)
#undef L1
#undef L2
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}
}  // namespace lbmx
