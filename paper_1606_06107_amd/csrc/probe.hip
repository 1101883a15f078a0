// Plain device copy (lbm_stream_copy in include/lbm.h): the memory-bandwidth
// reference the step kernels are compared with.  One 16-byte load and store
// per thread in a single pass over the buffer -- on MI355X the fastest of
// the simple copy shapes (grid-stride loops, several vectors per thread and
// non-temporal hints measured 4.5-5.8 TB/s for 2 GiB, this shape 6.2 TB/s).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <string>

#include "launch.hpp"
#include "lbm.h"

namespace lbmx {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream_copy(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                     size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace lbmx

extern "C" lbm_status lbm_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream) {
    if (!dst || !src) {
        lbmx::set_error("lbm_stream_copy: NULL buffer");
        return LBM_EINVAL;
    }
    if (bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16) {
        lbmx::set_error("lbm_stream_copy: size and addresses must be multiples of 16 bytes");
        return LBM_EINVAL;
    }
    const size_t n = bytes / 16;
    if (n == 0) return LBM_OK;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffu) {
        lbmx::set_error("lbm_stream_copy: buffer too large for one pass");
        return LBM_EINVAL;
    }
    hipLaunchKernelGGL(lbmx::k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                       (const lbmx::f32x4 *)src, (lbmx::f32x4 *)dst, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        lbmx::set_error((std::string("lbm_stream_copy: ") + hipGetErrorString(e)).c_str());
        return LBM_ELAUNCH;
    }
    return LBM_OK;
}
