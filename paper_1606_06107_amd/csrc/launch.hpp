// Internal launcher interface between the C-ABI host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmx {

// What a translational population buffer holds at time t (slot i of node x):
//   kLayoutPost     f*_i(x, t-1), post-collision: f_i(x, t) = slot i at S(x - c_i)
//   kLayoutStreamed f_i(x, t) itself (after initialisation; even in-place steps)
//   kLayoutSwapped  f*_i(x, t-1) kept in the opposite slot: f_i(x, t) = slot
//                   opp(i) at x - c_i (after an even in-place step)
enum { kLayoutPost = 0, kLayoutStreamed = 1, kLayoutSwapped = 2 };
// Step schemes: ping-pong (f_in -> f_out, output kLayoutPost), and the two
// halves of in-place streaming on periodic grids (f_in == f_out): even
// (kLayoutStreamed -> kLayoutSwapped: every access local, the result goes to
// the opposite slot) and odd (kLayoutSwapped -> kLayoutStreamed: gather slot
// opp(i) from x - c_i, scatter slot i to x + c_i; each node reads and writes
// the same set of locations, so nodes never conflict).
enum { kSchemePingPong = 0, kSchemeInPlaceEven = 1, kSchemeInPlaceOdd = 2 };

// Order of the values inside a translational buffer.  Plain: slot i of node
// x at i*N + x.  Blocked (3-D grids with n0 a multiple of 64): the nodes form
// blocks of 64 x-consecutive nodes (block b = x/64 in linear node order) and
// slot i of node x sits at ((x/64)*Q + i)*64 + x%64, so a block's populations
// are one contiguous run.  Rotational buffers are always plain.
constexpr int kBlk = 64;
__host__ __device__ inline size_t pop_index(int blocked, int Q, uint32_t N, int i, uint32_t x) {
    return blocked ? ((size_t)(x / kBlk) * Q + i) * kBlk + x % kBlk : (size_t)i * N + x;
}

// Arguments of the per-step kernels (one time step of Sec. V B).
struct StepArgs {
    const void *f_in;   // [Q][N] translational populations (see `layout`)
    const void *g_in;   // [7][N] rotational populations at time t
    void *f_out;        // [Q][N] translational populations after the step
    void *g_out;        // [7][N] rotational populations at time t+1
    int n0, n1, n2;     // nodes per axis
    int open0, open1, open2;  // 1 = open (clamp), 0 = periodic
    uint32_t N;         // n0*n1*n2
    int layout;         // kLayout* of f_in
    int scheme;         // kScheme*
    int blocked;        // value order of f_in / f_out (3-D only)
    double omega;       // 1/tau
    double n_rot;       // rotational degrees of freedom
    double *partials;   // NULL, or [ntiles][2+D] FP64 per-tile totals of time t
    int tiles0, tiles1, tiles2, ntiles;
    int reverse;        // 1: every XCD walks its band of tiles from the far end
};

// Arguments of the field/total/export kernels.
struct FieldArgs {
    const void *f;      // populations as stored
    const void *g;
    int n0, n1, n2, open0, open1, open2;
    uint32_t N;
    int layout;         // kLayout* of f
    int blocked;        // value order of f (f_out is always plain)
    double n_rot;
    double *rho, *u, *T;  // any may be NULL
    double *partials;     // NULL or [nblocks][2+D]
    void *f_out, *g_out;  // export targets (may be NULL)
    // Packed batches: node x belongs to tube t with offsets[t] <= x <
    // offsets[t+1] and uses n = n_rot_inst[t] instead of n_rot.
    const int64_t *offsets;
    const double *n_rot_inst;
    int num_inst;
};

struct InitArgs {
    const double *rho, *u, *T;
    void *f, *g;
    uint32_t N;
    int blocked;        // value order of f
};

// Copy plain populations src[Q][N] into dst in blocked order.
hipError_t launch_to_blocked(int dtype, int Q, uint32_t N, const void *src, void *dst, hipStream_t s);

// kind: lattice kind (kTensor, or kD2Q37 with dim 2; lbm_device.hpp).
hipError_t launch_init(int dtype, int dim, int kind, const InitArgs &a, hipStream_t s);
// Message returned by lbm_last_error() on this thread.
void set_error(const char *msg);
// tile = {tx, ty, tz}; returns hipErrorInvalidValue for a shape not compiled.
hipError_t launch_step(int dtype, int dim, int kind, const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_12_f32(int dim, const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_12_f64(int dim, const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_12_f32_inplace(int dim, const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_12_f64_inplace(int dim, const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_3(int dtype, const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_37_f32(const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_37_f64(const int tile[3], const StepArgs &a, hipStream_t s);

// Compiled tile shapes (nodes per workgroup along x, y).
#define LBMX_TILES_1D(X) X(64, 1) X(128, 1) X(256, 1) X(512, 1) X(1024, 1)
#define LBMX_TILES_2D(X) X(64, 4) X(32, 8) X(128, 2) X(256, 1) X(64, 8) X(32, 16) X(16, 16) X(64, 2)
#define LBMX_TILES_3D(X) X(64, 1) X(32, 2) X(16, 4)
#define LBMX_TILES_37(X) X(256, 1) X(128, 2) X(64, 2) X(64, 4) X(32, 8)
bool step_tile_supported(int dtype, int dim, int kind, const int tile[3]);
// Tiles (and therefore partial rows) of a step launch with this tile shape.
int step_ntiles(int dim, const int tile[3], int n0, int n1, int n2, int *t0, int *t1, int *t2);
// Fields and/or per-block partial totals; returns the number of blocks used.
hipError_t launch_fields(int dtype, int dim, int kind, const FieldArgs &a, int *nblocks, hipStream_t s);
hipError_t launch_export(int dtype, int dim, int kind, const FieldArgs &a, hipStream_t s);
// One time step with the rotational advection in m >= 2 sub-steps (ping-pong:
// a.f / a.g hold time t in a.layout, f_out receives the post-collision
// populations, g_out time t+1).  scratch: 17 N values of the population type.
hipError_t launch_step_sub(int dtype, int dim, int kind, const FieldArgs &a, void *f_out, void *g_out,
                           void *scratch, int m, double omega, hipStream_t s);
// Fixed-order sum of partials[nparts][K] into out[K] (one workgroup).
hipError_t launch_reduce(const double *partials, int nparts, int K, double *out, hipStream_t s);
// The same sum as row *slot of series[cap][K] (skipped if *slot >= cap);
// *slot then advances by one (device int64).
hipError_t launch_reduce_series(const double *partials, int nparts, int K, double *series, int64_t cap,
                                int64_t *slot, hipStream_t s);
// Quiet NaN into n values of dtype (a kernel: may be part of a graph).
hipError_t launch_fill_nan(int dtype, void *p, size_t n, hipStream_t s);
// *p = v on the stream (a kernel, so the write may be part of a graph).
hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t s);

}  // namespace lbmx
