// Instantiations and launcher of the 3-D (D3Q343) step kernels.
#include <hip/hip_runtime.h>

#include "step_impl.hpp"

namespace lbmx {

hipError_t launch_step_3(int dtype, const int tile[3], const StepArgs &a, hipStream_t s) {
    const dim3 grid(a.ntiles);
    bool done = false;
    if (a.blocked) {  // one 64-node block per tile
        if (tile[0] != kBlk || tile[1] != 1 || a.n0 % kBlk) return hipErrorInvalidValue;
        if (dtype == 0) hipLaunchKernelGGL((k_step_3<float, kBlk, 1, true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_step_3<double, kBlk, 1, true>), grid, dim3(256), 0, s, a);
        return hipGetLastError();
    }
#define L3(TXv, TYv)                                                                             \
    if (!done && tile[0] == TXv && tile[1] == TYv) {                                             \
        if (dtype == 0) hipLaunchKernelGGL((k_step_3<float, TXv, TYv, false>), grid, dim3(256), 0, s, a); \
        else hipLaunchKernelGGL((k_step_3<double, TXv, TYv, false>), grid, dim3(256), 0, s, a);  \
        done = true;                                                                             \
    }
    LBMX_TILES_3D(L3)
#undef L3
    if (!done) return hipErrorInvalidValue;
    return hipGetLastError();
}
}  // namespace lbmx
