// Memory-bandwidth references the step kernels are compared with (not part
// of the scheme):
//  - lbm_stream_copy: plain device copy.  One 16-byte load and store per
//    thread in a single pass over the buffer -- on MI355X the fastest of the
//    simple copy shapes (grid-stride loops, several vectors per thread and
//    non-temporal hints measured 4.5-5.8 TB/s for 2 GiB, this shape 6.2 TB/s).
//  - lbm_pattern_probe: the 2-D D2Q49 + D1Q7 step's memory pattern with no
//    arithmetic (49 translational rows gathered from the 7 x 7 neighbourhood
//    and stored, 7 rotational rows copied), in the three storage schemes;
//  - lbm_pattern_probe_3d: the same for the blocked 3-D D3Q343 step.
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

// One node per thread, 256 nodes of one grid row per workgroup.  Slot i has
// velocity (i % 7 - 3, i / 7 - 3); slot 48 - i has the opposite one.
//   MODE 0 ping-pong: fd[i](x) = fs[i](x - c_i), periodic wrap.
//   MODE 1 in place, even step: f[48 - i](x) = f[i](x).
//   MODE 2 in place, odd step: f[i](x + c_i) = f[48 - i](x - c_i)
//     (thread x reads and writes the same 49 locations, so no two threads
//     touch one location).
// POL 0: default cache policy; 1: non-temporal loads of f; 2: non-temporal
// loads and stores of f; 3: default for f, non-temporal loads and stores of
// g.  Otherwise g rows are copied with the default policy.
// BLK: f in 64-node blocks along x, population-major inside (value i of
// node (x, y) at ((y * nx / 64 + x / 64) * 49 + i) * 64 + x % 64; nx a
// multiple of 64) instead of rows [49][nx * ny].
template <int MODE, int POL, bool BLK>
__global__ void __launch_bounds__(256) k_pattern_2d(const float *fs, float *fd, const float *__restrict__ gs,
                                                   float *__restrict__ gd, int nx, int ny) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    const size_t N = (size_t)nx * ny;
    auto wrap = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
    auto at = [&](int i, int xx, int yy) {
        const size_t xw = (size_t)wrap(xx, nx), yw = (size_t)wrap(yy, ny);
        return BLK ? ((yw * (size_t)(nx / 64) + xw / 64) * 49 + i) * 64 + xw % 64 : (size_t)i * N + yw * nx + xw;
    };
    float v[49];
#pragma unroll
    for (int i = 0; i < 49; ++i) {
        const int cx = i % 7 - 3, cy = i / 7 - 3;
        const size_t src = MODE == 0 ? at(i, x - cx, y - cy) : MODE == 1 ? at(i, x, y) : at(48 - i, x - cx, y - cy);
        v[i] = POL == 1 || POL == 2 ? __builtin_nontemporal_load(fs + src) : fs[src];
    }
#pragma unroll
    for (int i = 0; i < 49; ++i) {
        const int cx = i % 7 - 3, cy = i / 7 - 3;
        const size_t dst = MODE == 0 ? at(i, x, y) : MODE == 1 ? at(48 - i, x, y) : at(i, x + cx, y + cy);
        if (POL == 2)
            __builtin_nontemporal_store(v[i], fd + dst);
        else
            fd[dst] = v[i];
    }
    const size_t o = (size_t)y * nx + x;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        if (POL == 3)
            __builtin_nontemporal_store(__builtin_nontemporal_load(gs + (size_t)j * N + o), gd + (size_t)j * N + o);
        else
            gd[(size_t)j * N + o] = gs[(size_t)j * N + o];
    }
}

template <int MODE, bool BLK>
static void launch_pattern(int pol, dim3 grid, hipStream_t s, const float *fs, float *fd, const float *gs, float *gd,
                           int nx, int ny) {
    if (pol == 0)
        hipLaunchKernelGGL((k_pattern_2d<MODE, 0, BLK>), grid, dim3(256), 0, s, fs, fd, gs, gd, nx, ny);
    else if (pol == 1)
        hipLaunchKernelGGL((k_pattern_2d<MODE, 1, BLK>), grid, dim3(256), 0, s, fs, fd, gs, gd, nx, ny);
    else if (pol == 2)
        hipLaunchKernelGGL((k_pattern_2d<MODE, 2, BLK>), grid, dim3(256), 0, s, fs, fd, gs, gd, nx, ny);
    else
        hipLaunchKernelGGL((k_pattern_2d<MODE, 3, BLK>), grid, dim3(256), 0, s, fs, fd, gs, gd, nx, ny);
}

// The 3-D D3Q343 + D1Q7 step's memory pattern in the blocked order (64
// x-consecutive nodes per block, population-major inside: value i of node
// (x, y, z) at ((b * 343 + i) * 64 + x % 64, b the node's block), ping-pong:
// fd[i](x) = fs[i](x - c_i) periodically, c_i = (i % 7 - 3, i / 7 % 7 - 3,
// i / 49 - 3).  One workgroup per block, four waves, wave w moving
// populations 86 w .. 86 w + 85 (all loaded, then all stored, as the step
// kernel does); wave 0 also copies the 7 rotational rows [7][N] of its nodes.
template <int N_> struct IntC { static constexpr int value = N_; };
template <int B, int E, typename F> __device__ __forceinline__ void for_range(F &&f) {
    if constexpr (B < E) {
        f(IntC<B>{});
        for_range<B + 1, E>(f);
    }
}

// Wave W of a block moves populations 86 W .. min(343, 86 W + 86): addresses
// as the step kernel forms them -- a lane offset per c_x (the source node's
// block and lane), a wave-uniform base per (c_y, c_z) source row, the
// population number a constant.
template <int POL, int W>
__device__ __forceinline__ void move_3d(const float *fs, float *fd, int n0, int n1, int n2, int x, int y, int z,
                                        int l, size_t dst_base) {
    constexpr int Q = 343, I0 = 86 * W, I1 = (86 * W + 86 < Q) ? 86 * W + 86 : Q;
    const int nb0 = n0 / 64;
    auto wrap = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
    size_t xo[7];  // element offset of (x - c_x) within its row of blocks, population 0
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const int xs = wrap(x - (k - 3), n0);
        xo[k] = (size_t)(xs / 64) * Q * 64 + xs % 64;
    }
    float v[I1 - I0];
    for_range<I0, I1>([&](auto I) {
        constexpr int i = decltype(I)::value, cx = i % 7 - 3, cy = i / 7 % 7 - 3, cz = i / 49 - 3;
        const size_t row = ((size_t)wrap(z - cz, n2) * n1 + wrap(y - cy, n1)) * nb0 * Q * 64;  // uniform
        const float *p = fs + row + xo[cx + 3] + (size_t)i * 64;
        v[i - I0] = POL == 1 || POL == 2 ? __builtin_nontemporal_load(p) : *p;
    });
    for_range<I0, I1>([&](auto I) {
        constexpr int i = decltype(I)::value;
        float *p = fd + dst_base + (size_t)i * 64;
        if constexpr (POL == 2)
            __builtin_nontemporal_store(v[i - I0], p);
        else
            *p = v[i - I0];
    });
}

// The 3-D D3Q343 + D1Q7 step's memory pattern in the blocked order (64
// x-consecutive nodes per block, population-major inside: value i of node
// (x, y, z) at (b * 343 + i) * 64 + x % 64, b the node's block), ping-pong:
// fd[i](x) = fs[i](x - c_i) periodically, c_i = (i % 7 - 3, i / 7 % 7 - 3,
// i / 49 - 3).  One workgroup per block, four waves, each moving its quarter
// of the populations (all loaded, then all stored, as the step kernel does);
// wave 0 also copies the 7 rotational rows [7][N] of its nodes.
template <int POL>
__global__ void __launch_bounds__(256) k_pattern_3d(const float *fs, float *fd, const float *__restrict__ gs,
                                                   float *__restrict__ gd, int n0, int n1, int n2) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int nb0 = n0 / 64;
    const int bx = (int)(blockIdx.x % (unsigned)nb0);
    const int yz = (int)(blockIdx.x / (unsigned)nb0);
    const int y = yz % n1, z = yz / n1;
    const int x = 64 * bx + l;
    const size_t dst_base = (size_t)blockIdx.x * 343 * 64 + l;
    if (w == 0)
        move_3d<POL, 0>(fs, fd, n0, n1, n2, x, y, z, l, dst_base);
    else if (w == 1)
        move_3d<POL, 1>(fs, fd, n0, n1, n2, x, y, z, l, dst_base);
    else if (w == 2)
        move_3d<POL, 2>(fs, fd, n0, n1, n2, x, y, z, l, dst_base);
    else
        move_3d<POL, 3>(fs, fd, n0, n1, n2, x, y, z, l, dst_base);
    if (w == 0) {
        const size_t N = (size_t)n0 * n1 * n2, o = ((size_t)z * n1 + y) * n0 + x;
#pragma unroll
        for (int j = 0; j < 7; ++j) gd[(size_t)j * N + o] = gs[(size_t)j * N + o];
    }
}

}  // namespace lbmx

extern "C" lbm_status lbm_pattern_probe_3d(int32_t policy, float *f_dst, const float *f_src, float *g_dst,
                                           const float *g_src, int32_t n0, int32_t n1, int32_t n2,
                                           void *hip_stream) {
    if (!f_dst || !f_src || !g_dst || !g_src) {
        lbmx::set_error("lbm_pattern_probe_3d: NULL buffer");
        return LBM_EINVAL;
    }
    if (policy < 0 || policy > 2) {
        lbmx::set_error("lbm_pattern_probe_3d: policy must be 0, 1 or 2");
        return LBM_EINVAL;
    }
    if (f_dst == f_src || g_dst == g_src) {
        lbmx::set_error("lbm_pattern_probe_3d: source and destination buffers must be distinct");
        return LBM_EINVAL;
    }
    if (n0 < 64 || n0 % 64 || n1 < 4 || n2 < 4 || (int64_t)n0 * n1 * n2 * 4 >= ((int64_t)1 << 32)) {
        lbmx::set_error("lbm_pattern_probe_3d: need n0 a multiple of 64, n1, n2 >= 4, n0 n1 n2 * 4 < 2^32");
        return LBM_EINVAL;
    }
    const dim3 grid((unsigned)((int64_t)n0 / 64 * n1 * n2));
    const hipStream_t s = (hipStream_t)hip_stream;
    if (policy == 0)
        hipLaunchKernelGGL((lbmx::k_pattern_3d<0>), grid, dim3(256), 0, s, f_src, f_dst, g_src, g_dst, n0, n1, n2);
    else if (policy == 1)
        hipLaunchKernelGGL((lbmx::k_pattern_3d<1>), grid, dim3(256), 0, s, f_src, f_dst, g_src, g_dst, n0, n1, n2);
    else
        hipLaunchKernelGGL((lbmx::k_pattern_3d<2>), grid, dim3(256), 0, s, f_src, f_dst, g_src, g_dst, n0, n1, n2);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        lbmx::set_error((std::string("lbm_pattern_probe_3d: ") + hipGetErrorString(e)).c_str());
        return LBM_ELAUNCH;
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_pattern_probe(int32_t mode, int32_t policy, float *f_dst, const float *f_src,
                                        float *g_dst, const float *g_src, int32_t nx, int32_t ny,
                                        void *hip_stream) {
    if (!f_dst || !f_src || !g_dst || !g_src) {
        lbmx::set_error("lbm_pattern_probe: NULL buffer");
        return LBM_EINVAL;
    }
    if (mode < 0 || mode > 5 || policy < 0 || policy > 3) {
        lbmx::set_error("lbm_pattern_probe: mode must be 0 to 5 and policy 0 to 3");
        return LBM_EINVAL;
    }
    const bool blk = mode >= 3;
    if (blk && nx % 64) {
        lbmx::set_error("lbm_pattern_probe: the blocked modes need nx a multiple of 64");
        return LBM_EINVAL;
    }
    if ((mode % 3 == 0) == (f_dst == f_src) || g_dst == g_src) {
        lbmx::set_error("lbm_pattern_probe: mode 0 needs distinct f buffers, modes 1 and 2 one buffer; "
                        "g buffers must be distinct");
        return LBM_EINVAL;
    }
    if (nx < 4 || ny < 4 || ny > 65535 || (int64_t)nx * ny * 49 >= (int64_t)1 << 40) {
        lbmx::set_error("lbm_pattern_probe: need 4 <= nx, 4 <= ny <= 65535");
        return LBM_EINVAL;
    }
    const dim3 grid((unsigned)((nx + 255) / 256), (unsigned)ny);
    const hipStream_t s = (hipStream_t)hip_stream;
    if (mode == 0)
        lbmx::launch_pattern<0, false>(policy, grid, s, f_src, f_dst, g_src, g_dst, nx, ny);
    else if (mode == 1)
        lbmx::launch_pattern<1, false>(policy, grid, s, f_src, f_dst, g_src, g_dst, nx, ny);
    else if (mode == 2)
        lbmx::launch_pattern<2, false>(policy, grid, s, f_src, f_dst, g_src, g_dst, nx, ny);
    else if (mode == 3)
        lbmx::launch_pattern<0, true>(policy, grid, s, f_src, f_dst, g_src, g_dst, nx, ny);
    else if (mode == 4)
        lbmx::launch_pattern<1, true>(policy, grid, s, f_src, f_dst, g_src, g_dst, nx, ny);
    else
        lbmx::launch_pattern<2, true>(policy, grid, s, f_src, f_dst, g_src, g_dst, nx, ny);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        lbmx::set_error((std::string("lbm_pattern_probe: ") + hipGetErrorString(e)).c_str());
        return LBM_ELAUNCH;
    }
    return LBM_OK;
}

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
