// Finite-difference update of the translational populations (Sec. V A
// written for f as well: forward Euler in time, third-order upwind in space,
// BGK), as an alternative to collide-and-stream.  Interface between the
// C-ABI host code and the kernels of step_fd.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmx {

struct FdArgs {
    const void *f_in;   // [Q][N] translational populations at time t (values at their nodes)
    const void *g_in;   // [7][N] rotational populations at time t
    void *f_out;        // [Q][N] at time t + dt
    void *g_out;        // [7][N] at time t + dt
    int n0, n1;         // nodes per axis (n1 = 1 in 1-D)
    int open0, open1;   // 1 = open (clamp), 0 = periodic
    uint32_t N;
    double lambda;      // time step in units of the streaming step 1/r (Courant factor)
    double omega;       // lambda / tau: collision rate per step
    double n_rot;
    int tiles0, ntiles;
};

// dim 1 (D1Q7) or 2 (kind: kTensor = D2Q49, kD2Q37); tile = 256 x 1 (1-D)
// or 64 x 4 (2-D).  hipErrorInvalidValue for other combinations.
hipError_t launch_step_fd(int dtype, int dim, int kind, const FdArgs &a, hipStream_t s);
// Tile of the finite-difference kernels along x and y.
void fd_tile(int dim, int *tx, int *ty);

}  // namespace lbmx
