// Internal launcher interface between the C-ABI host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmx {

// Arguments of the per-step kernels (one time step of Sec. V B).
struct StepArgs {
    const void *f_in;   // [Q][N] translational populations (see `streamed`)
    const void *g_in;   // [7][N] rotational populations at time t
    void *f_out;        // [Q][N] post-collision translational populations
    void *g_out;        // [7][N] rotational populations at time t+1
    int n0, n1, n2;     // nodes per axis
    int open0, open1, open2;  // 1 = open (clamp), 0 = periodic
    uint32_t N;         // n0*n1*n2
    int streamed;       // 1: f_in holds streamed populations f(t) (read in place);
                        // 0: f_in holds post-collision f*(t-1) (gathered from x - c)
    double omega;       // 1/tau
    double n_rot;       // rotational degrees of freedom
    double *partials;   // NULL, or [ntiles][2+D] FP64 per-tile totals of time t
    int tiles0, tiles1, tiles2, ntiles;
};

// Arguments of the field/total/export kernels.
struct FieldArgs {
    const void *f;      // populations as stored
    const void *g;
    int n0, n1, n2, open0, open1, open2;
    uint32_t N;
    int streamed;
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
};

hipError_t launch_init(int dtype, int dim, const InitArgs &a, hipStream_t s);
// Message returned by lbm_last_error() on this thread.
void set_error(const char *msg);
// tile = {tx, ty, tz}; returns hipErrorInvalidValue for a shape not compiled.
hipError_t launch_step(int dtype, int dim, const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_12_f32(int dim, const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_12_f64(int dim, const int tile[3], const StepArgs &a, hipStream_t s);
hipError_t launch_step_3(int dtype, const int tile[3], const StepArgs &a, hipStream_t s);

// Compiled tile shapes (nodes per workgroup along x, y).
#define LBMX_TILES_1D(X) X(64, 1) X(128, 1) X(256, 1) X(512, 1) X(1024, 1)
#define LBMX_TILES_2D(X) X(64, 4) X(32, 8) X(128, 2) X(256, 1) X(64, 8) X(32, 16) X(16, 16) X(64, 2)
#define LBMX_TILES_3D(X) X(64, 1) X(32, 2) X(16, 4)
bool step_tile_supported(int dtype, int dim, const int tile[3]);
// Tiles (and therefore partial rows) of a step launch with this tile shape.
int step_ntiles(int dim, const int tile[3], int n0, int n1, int n2, int *t0, int *t1, int *t2);
// Fields and/or per-block partial totals; returns the number of blocks used.
hipError_t launch_fields(int dtype, int dim, const FieldArgs &a, int *nblocks, hipStream_t s);
hipError_t launch_export(int dtype, int dim, const FieldArgs &a, hipStream_t s);
// Fixed-order sum of partials[nparts][K] into out[K] (one workgroup).
hipError_t launch_reduce(const double *partials, int nparts, int K, double *out, hipStream_t s);

}  // namespace lbmx
