/*
 * lbm.h -- C ABI of liblbmx, an MI355X (gfx950) implementation of the
 * decoupled Hermite-expansion lattice Boltzmann scheme for compressible flow
 * with arbitrary specific heat ratio (Hu, Zhang & Geng, arXiv:1606.06107).
 *
 * The scheme (Secs. II-V of the paper) advances two population sets per node:
 *   f_i  translational populations (the paper's g_i) on a Gauss-Hermite
 *        lattice: D1Q7, or its tensor powers D2Q49, D3Q343 (Table II, Sec. IV).
 *        Streamed with xi_i = r c_i: collide, then shift by the integer c_i.
 *   g_j  rotational populations (the paper's h_j) on D1Q7, eta_j = r j:
 *        advected with the fluid velocity u by the third-order upwind
 *        difference of Sec. V A with forward-Euler time stepping, and relaxed.
 * Both relax with BGK (omega = 1/tau, tau in time steps) towards the
 * fourth-order Hermite equilibria of Sec. IV evaluated at the node's
 * (rho, u, T).  T comes from the total energy with D+n degrees of freedom
 * (Sec. V B step 4), so gamma = (D+n+2)/(D+n) (Sec. III).
 * Units are the paper's dimensionless ones (T0 = R_g = 1).  A step moves a
 * population c_i nodes, i.e. dt = dx / r; the rotational Courant number along
 * axis a is u_a / r.
 *
 * Conventions shared by every entry point
 *  - Every call returns lbm_status (LBM_OK = 0) and never throws or aborts.
 *    On failure lbm_last_error() returns a message (thread-local).
 *  - Every pointer argument named f, g, rho, u, T, totals, offsets, ... is a
 *    DEVICE pointer, allocated and owned by the caller (e.g. a torch tensor);
 *    it must stay valid while any handle or launch uses it.  The library owns
 *    only host-side handles and the HIP graphs it instantiates.
 *  - Work is enqueued asynchronously on the caller's HIP stream (hipStream_t
 *    passed as void*; NULL = the null stream).  The host sees argument and
 *    launch errors only; numerical failure (non-finite values, rho <= 0,
 *    T <= 0) is reported in device memory (totals, status) that the caller
 *    reads after synchronising the stream.
 *  - Population arrays are structure-of-arrays [Q][N], node index x fastest:
 *    node(x,y,z) = x + nx*(y + ny*z).  Lattice direction i of D1Q7^D is
 *    i = cx+3 (1-D), (cy+3)*7 + cx+3 (2-D), ((cz+3)*7 + cy+3)*7 + cx+3 (3-D).
 *  - Macroscopic fields are FP64: rho[N], u[D][N], T[N].
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2

typedef int32_t lbm_status;
enum {
    LBM_OK = 0,
    LBM_EINVAL = 1,       /* invalid argument or descriptor */
    LBM_EDEVICE = 2,      /* no usable gfx950 device, or a HIP runtime error */
    LBM_ENOMEM = 3,       /* host allocation failed */
    LBM_EUNSUPPORTED = 4, /* valid but not implemented combination */
    LBM_ELAUNCH = 5       /* kernel launch or graph error */
};

/* Translational lattices: D1Q7 (Table II) and its tensor powers, and the
 * D2Q37 set of Table I (the D2Q49 velocities without the groups (2r,2r) and
 * (3r,2r), one weight per group, at the D1Q7 r; dim 2). */
enum { LBM_D1Q7 = 1, LBM_D2Q49 = 2, LBM_D3Q343 = 3, LBM_D2Q37 = 4 };
/* Population storage type. */
enum { LBM_F32 = 0, LBM_F64 = 1 };
/* Boundary condition per axis: periodic wrap, or open (zero-gradient clamp
 * of the streaming source index and of the upwind stencil; Sec. VI uses open
 * left/right ends). */
enum { LBM_BC_PERIODIC = 0, LBM_BC_OPEN = 1 };

typedef struct {
    int32_t abi_version; /* must equal LBM_ABI_VERSION */
    int32_t dim;         /* spatial dimension D: 1, 2 or 3 (must match lattice) */
    int64_t n[3];        /* nodes per axis; unused axes must be 1.  Periodic axes
                            need n >= 3; N = n0*n1*n2 with N * sizeof(pop) < 2^32 */
    int32_t lattice;     /* LBM_D1Q7 (dim 1), LBM_D2Q49 or LBM_D2Q37 (dim 2),
                            LBM_D3Q343 (dim 3); Q = 7, 49, 37, 343 */
    int32_t dtype;       /* LBM_F32 or LBM_F64 population storage */
    int32_t bc[3];       /* LBM_BC_PERIODIC or LBM_BC_OPEN per axis */
    double n_rot;        /* rotational degrees of freedom n >= 0 (real);
                            gamma = (D+n+2)/(D+n) */
    double tau;          /* BGK relaxation time in time steps, tau > 0.5 */
    int32_t g_substeps;  /* 0 or 1: the rotational update of Sec. V A as written
                            (one forward-Euler upwind step with Courant number
                            u_a / r).  m in [2, 64]: its advection in m sub-steps
                            of Courant number u_a / (m r), relaxation once per
                            step -- the update is linearly unstable beyond a
                            Courant number that falls with 1/tau (0.67 at tau =
                            1, 0.375 at tau = 2/3), which strong shocks exceed.
                            Runs a plain one-node-per-thread path, ping-pong
                            only (no in-place streaming, no finite-difference
                            update), with 17 N population values of extra
                            workspace */
    void *f[2];          /* two device buffers of Q*N values of dtype (ping-pong);
                            with in-place streaming (lbm_set_inplace) only f[0]
                            is used, but both must be given.  The order of the
                            values inside is the library's (lbm_set_blocked):
                            read and write populations through
                            lbm_populations / lbm_init_populations */
    void *g[2];          /* two device buffers [7][N] of dtype (ping-pong) */
    void *workspace;     /* device scratch of lbm_workspace_bytes() bytes, 256-B
                            aligned (reduction partials, the monitor's row
                            counter, sub-step buffers); caller-owned */
} lbm_desc;

typedef struct lbm_sim_s *lbm_sim; /* opaque host handle; owns no device memory */

/* Bytes of device workspace a descriptor needs (0 on an invalid descriptor). */
size_t lbm_workspace_bytes(const lbm_desc *desc);

/* Validate desc, create a handle bound to hip_stream and set every node to
 * equilibrium: f = f^eq(rho, u, T), g = g^eq(T) (Sec. IV), written to f[0],
 * g[0].  rho[N], u[D][N], T[N]: device FP64 fields.  Time is 0 afterwards.
 * Errors: LBM_EINVAL (descriptor, NULL pointers), LBM_EDEVICE, LBM_ELAUNCH. */
lbm_status lbm_init(const lbm_desc *desc, const double *rho, const double *u,
                    const double *T, void *hip_stream, lbm_sim *out);

/* As lbm_init, but the state at time 0 is given as populations: f0[Q][N] and
 * g0[7][N] of the descriptor's dtype, copied into f[0], g[0] (device). */
lbm_status lbm_init_populations(const lbm_desc *desc, const void *f0, const void *g0,
                                void *hip_stream, lbm_sim *out);

/* Advance nsteps >= 0 time steps (Sec. V B steps 1-5, one fused kernel per
 * step: gather of the streamed f, FP64 moments and temperature, Hermite
 * equilibria, BGK, upwind advection of g, boundary conditions).  With graphs
 * enabled (default) and nsteps > 1 the steps replay as one HIP graph.
 * Errors: LBM_EINVAL, LBM_ELAUNCH. */
lbm_status lbm_step(lbm_sim sim, int64_t nsteps);

/* Record and instantiate, without running it, the HIP graph that
 * lbm_step(sim, nsteps) replays from the current state, so that the later
 * lbm_step call only launches it (capture and instantiation take host time,
 * and allocate; callers that time or serve steps do them ahead).  A graph
 * is reused by any lbm_step of the same length that starts from a state with
 * the same buffer parity, streaming layout, tile and monitor settings and
 * the same phase t mod every of the monitor (the row a monitored step fills
 * comes from a counter in the workspace, not from the recorded time).  Up
 * to 8 graphs are kept per handle.  No-op when graphs are disabled or
 * nsteps <= 1.  Errors: LBM_EINVAL, LBM_EUNSUPPORTED, LBM_ELAUNCH. */
lbm_status lbm_prepare(lbm_sim sim, int64_t nsteps);

/* Fields and conservation totals at the current time.  rho[N], u[D][N], T[N]
 * and totals[2+D] = {mass, momentum_0..D-1, energy} (energy = sum over nodes
 * of E_t + rho e_r, i.e. rho (|u|^2/2 + (D+n)T/2)), all device FP64; any may
 * be NULL to skip.  Moments are accumulated in FP64 from the populations and
 * T is extracted in FP64 (Sec. V B steps 3-4); totals use a deterministic
 * fixed-order two-stage reduction. */
lbm_status lbm_moments(lbm_sim sim, double *rho, double *u, double *T, double *totals);

/* Populations at the current time in canonical form (streamed translational
 * populations f(t), rotational g(t)), written to device buffers f_out[Q][N],
 * g_out[7][N] of the descriptor's dtype; either may be NULL. */
lbm_status lbm_populations(lbm_sim sim, void *f_out, void *g_out);

/* Record conservation totals every `every` steps during lbm_step, fused into
 * the step kernel: row k of series[capacity][2+D] (device FP64) receives the
 * totals of time t with t = k*every (t counted from lbm_init).  Steps whose
 * row is >= capacity record nothing.  every = 0 switches recording off.
 * The next row to fill is kept in the workspace (set here, on the sim's
 * stream), so the workspace must not be shared by two handles that record
 * at the same time. */
lbm_status lbm_set_monitor(lbm_sim sim, int64_t every, double *series, int64_t capacity);

/* Time-step counter since lbm_init. */
lbm_status lbm_time(lbm_sim sim, int64_t *t);

/* Debug flags.  LBM_DEBUG_POISON: before every step, fill the buffers the
 * step writes without reading them (the rotational destination; with
 * ping-pong streaming the translational one too) with quiet NaN, so that a
 * population the step fails to write shows up as NaN in the next step's
 * fields.  Same results otherwise; one extra fill per step.  0 turns them off.
 * Errors: LBM_EINVAL. */
enum { LBM_DEBUG_POISON = 1 };
lbm_status lbm_set_debug(lbm_sim sim, int32_t flags);

/* Enable (1) or disable (0) HIP-graph replay of multi-step calls. */
lbm_status lbm_set_graphs(lbm_sim sim, int32_t enable);

/* Streaming scheme of the translational populations, chosen before the
 * first step (right after lbm_init / lbm_init_populations).  enable = 0:
 * ping-pong between f[0] and f[1] (pull from the post-collision values of the
 * previous step).  enable = 1: in place in f[0] -- even steps read and write
 * every node's own populations, storing direction i in the slot of -c_i; odd
 * steps read those slots from x - c_i and write slot i at x + c_i (each node
 * reads and writes the same set of locations).  Same arithmetic, identical
 * results, half the translational memory; at 1024^2 FP32 the single buffer
 * largely stays in the memory-side cache.  Default: in place when every axis
 * is periodic and dim <= 2.  Errors: LBM_EINVAL (after the first step),
 * LBM_EUNSUPPORTED (enable on an open axis or in 3-D). */
lbm_status lbm_set_inplace(lbm_sim sim, int32_t enable);

/* Update of the translational populations, chosen before the first step.
 * courant = 0 (default): collide and stream (exact shift by the integer
 * lattice velocity; time step dx / r).  0 < courant <= 1: the
 * finite-difference form of Sec. V A for f as well as g -- forward Euler in
 * time, third-order upwind in space, BGK -- with time step courant * dx / r,
 * so population i moves with Courant number courant * c_i per axis; tau
 * stays in units of dx / r (collision rate courant / tau per step).  The
 * scheme amplifies some mode at every step size (weakly below courant ~
 * 1/6, by > 4x per step at courant = 1 for |c| = 3); the collisions keep
 * e.g. the Sec. VI tube bounded at courant <= 0.2.  1-D and 2-D grids
 * (D1Q7, D2Q49, D2Q37), ping-pong (in-place streaming off); no conservation
 * monitor; each lbm_step advances steps of courant * dx / r.  Errors:
 * LBM_EINVAL (after the first step, courant outside [0, 1]),
 * LBM_EUNSUPPORTED (3-D). */
lbm_status lbm_set_fd(lbm_sim sim, double courant);

/* Order of the translational values inside f[0], f[1], chosen before the
 * first step.  enable = 0: plain [Q][N] (slot i of node x at i*N + x).
 * enable = 1 (3-D grids with n0 a multiple of 64): blocks of 64 x-consecutive
 * nodes, slot i of node x at ((x/64)*Q + i)*64 + x%64, so the 343 populations
 * of one workgroup tile are one contiguous run (the step writes each block
 * in one piece and reads 49 source rows instead of 343 separate streams).
 * Same arithmetic, identical results.  Switching reorders the current state
 * into the other f buffer on the sim's stream; enabling sets the tile to
 * 64x1x1, the only one the blocked step runs with.  Default: blocked where
 * possible.  Errors: LBM_EINVAL (after the first step), LBM_EUNSUPPORTED
 * (enable on a grid that cannot be blocked), LBM_ELAUNCH. */
lbm_status lbm_set_blocked(lbm_sim sim, int32_t enable);

/* Launch shape of the step kernel: nodes per workgroup tile along x, y, z
 * (product 64..1024, a multiple of 64; tile_x a multiple of 16).  Used by the
 * autotuner; results do not depend on it.  LBM_EUNSUPPORTED if the shape is
 * not compiled, or not 64x1x1 under the blocked order.  (The finite-difference
 * update of lbm_set_fd runs with its own fixed shape.) */
lbm_status lbm_set_tile(lbm_sim sim, int32_t tx, int32_t ty, int32_t tz);

/* Release the handle and its graphs (NULL-safe).  Device buffers are the
 * caller's. */
lbm_status lbm_destroy(lbm_sim sim);

/* Message of the last failed call on this thread ("" if none). */
const char *lbm_last_error(void);

/* Plain device-to-device copy of `bytes` (a multiple of 16; both buffers
 * 16-byte aligned) on hip_stream: one 16-byte load and store per thread in
 * one pass.  Not part of the scheme: the measured memory-bandwidth reference
 * that the step kernels' achieved bandwidth is set against (the HBM peak of
 * the data sheet is not reached by any copy).  Errors: LBM_EINVAL,
 * LBM_ELAUNCH. */
lbm_status lbm_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Memory pattern of the 2-D D2Q49 + D1Q7 FP32 step with no arithmetic, on an
 * nx x ny periodic grid (4 <= nx, 4 <= ny <= 65535): 49 translational rows
 * f[49][nx*ny] and 7 rotational rows g[7][nx*ny] (x fastest), device
 * buffers.  Slot i has velocity (i % 7 - 3, i / 7 - 3), slot 48 - i the
 * opposite.  mode 0 (ping-pong, f_dst != f_src): f_dst[i](x) =
 * f_src[i](x - c_i); mode 1 (in place, even step, f_dst == f_src):
 * f[48 - i](x) = f[i](x); mode 2 (in place, odd step, f_dst == f_src):
 * f[i](x + c_i) = f[48 - i](x - c_i); modes 3, 4, 5: the same with f in
 * 64-node blocks along x (value i of node (x, y) at
 * ((y * nx / 64 + x / 64) * 49 + i) * 64 + x % 64; nx a multiple of 64).
 * Every mode copies g_src to g_dst
 * (distinct).  policy 0: default cache policy; 1: non-temporal loads of f;
 * 2: non-temporal loads and stores of f; 3: default policy for f,
 * non-temporal loads and stores of g.  448 B of memory traffic per node,
 * as the step.  Not part of the scheme: the pattern's bandwidth ceiling that
 * the step kernels are set against.  Errors: LBM_EINVAL, LBM_ELAUNCH. */
lbm_status lbm_pattern_probe(int32_t mode, int32_t policy, float *f_dst, const float *f_src, float *g_dst,
                             const float *g_src, int32_t nx, int32_t ny, void *hip_stream);

/* Memory pattern of the 3-D D3Q343 + D1Q7 FP32 step in the blocked order, no
 * arithmetic, ping-pong, on an n0 x n1 x n2 periodic grid (n0 a multiple of
 * 64, n1, n2 >= 4, n0 n1 n2 * 4 < 2^32): f [343][N] values in 64-node blocks
 * (value i of node (x, y, z) at ((b * 343 + i) * 64 + x % 64), b = (z n1 +
 * y) n0 / 64 + x / 64), f_dst[i](x) = f_src[i](x - c_i) with c_i =
 * (i % 7 - 3, i / 7 % 7 - 3, i / 49 - 3); g [7][N] (x fastest) copied.  policy
 * 0: default cache policy; 1: non-temporal loads of f; 2: non-temporal loads
 * and stores of f.  2800 B of memory traffic per node, as the step.  Not
 * part of the scheme: the bandwidth ceiling of that pattern.  Errors:
 * LBM_EINVAL, LBM_ELAUNCH. */
lbm_status lbm_pattern_probe_3d(int32_t policy, float *f_dst, const float *f_src, float *g_dst,
                                const float *g_src, int32_t n0, int32_t n1, int32_t n2, void *hip_stream);

/* Lattice constants the library computes with: Q, r, and (if not NULL) the
 * weights w[Q] and velocities c[Q][3] (integers) of the population slots in
 * storage order (populations[Q][N] of lbm_populations / lbm_init_populations;
 * slot Q-1-i holds -c_i).  Host pointers. */
lbm_status lbm_lattice_info(int32_t lattice, int32_t *Q, double *r, double *w, int32_t *c);

/* ------------------------------------------------------------------------ */
/* Batched 1-D shock tubes: one persistent launch advances many independent  */
/* D1Q7 + D1Q7 tubes of uneven length, each with its own n, tau and number   */
/* of steps, both ends open (Sec. VI boundary treatment).                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t abi_version;    /* LBM_ABI_VERSION */
    int32_t dtype;          /* LBM_F32 or LBM_F64 */
    int64_t num_instances;  /* I >= 1 */
    int64_t total_nodes;    /* sum of lengths = offsets[I] < 2^31 */
    const int64_t *offsets; /* device [I+1], offsets[0] = 0, increasing; tube i
                               owns packed nodes offsets[i] .. offsets[i+1]-1,
                               length >= 4 */
    const double *n_rot;    /* device [I], n >= 0 */
    const double *tau;      /* device [I], tau > 0.5 */
    const int64_t *nsteps;  /* device [I], steps to advance in lbm_batch_step, >= 0 */
    void *f[2];             /* device [7][total] of dtype: f[0] holds the state,
                               f[1] is scratch */
    void *g[2];             /* device [7][total] of dtype: same roles */
    int32_t *status;        /* device [I] out: 0 ok, 1 non-finite, 2 rho<=0 or T<=0,
                               3 empty tube, 4 not completed (a bounded wait of
                               the long-tube work queue gave up; not expected);
                               a failing tube stops at the step that failed and
                               its state is then unspecified */
    int64_t *steps_done;    /* device [I] out (may be NULL): steps completed */
    void *workspace;        /* device, lbm_batch_workspace_bytes() bytes */
    int32_t block;          /* threads per workgroup: 256, 512 or 1024 (0 = default) */
    int32_t chunk;          /* nodes per on-chip chunk, 0 = largest that fits */
    int32_t superstep;      /* time steps per on-chip pass of a chunked tube
                               (0 = default 24, fewer if the halo of the
                               sub-steps below does not leave room) */
    int32_t g_substeps;     /* as lbm_desc.g_substeps, for every tube: 0 or 1 =
                               the rotational update as written; m in [2, 64]
                               = its advection in m sub-steps of Courant number
                               u / (m r), the relaxation once per step (chunk
                               halos grow to max(3, 2m) nodes per step) */
} lbm_batch_desc;

size_t lbm_batch_workspace_bytes(const lbm_batch_desc *desc);

/* Equilibrium initial state of every tube from packed FP64 fields rho[total],
 * u[total], T[total] (device). */
lbm_status lbm_batch_init(const lbm_batch_desc *desc, const double *rho, const double *u,
                          const double *T, void *hip_stream);

/* Advance every tube i by nsteps[i] steps in ONE persistent launch (one
 * workgroup per compute unit).  Tubes longer than one on-chip chunk advance
 * in passes of at most `superstep` steps: each pass cuts such a tube into
 * chunks with overlapping halos, and the chunks go through a device work
 * queue shared by all workgroups; the workgroup that completes a tube's
 * pass queues the next one (a failed tube stops there).  Workgroups that
 * find the queue empty, and all of them once the long tubes are done, take
 * the tubes that fit on chip, which run their whole time loop there,
 * longest work first.  The result is left in f[0], g[0]; status[i] is
 * written by the end of the launch.  A tube with nsteps[i] = 0 is not read
 * or written (status 0, 3 if empty; steps 0), so a call that advances a few
 * tubes of a large batch costs only their work. */
lbm_status lbm_batch_step(const lbm_batch_desc *desc, void *hip_stream);

/* For callers that cannot allocate device memory or instantiate graphs
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): lbm_batch_step without a workspace.  desc->workspace is
 * ignored (may be NULL); the launch uses a fixed 8 MiB device array of the
 * library instead, one per device, held until the process ends.  The
 * schedule kernel re-initialises every word of it that the launch reads, so
 * the previous call's contents do not matter; but every call on one device
 * shares the array, so calls that overlap in time on one device (different
 * streams, or threads) race and must be serialised by the caller.  The two
 * kernels are launched directly on hip_stream (no graph); no hipMalloc,
 * hipFree or graph instantiation happens.  Results are those of
 * lbm_batch_step on the same descriptor, bitwise.  Errors: LBM_EINVAL (as
 * lbm_batch_step, or lbm_batch_workspace_bytes(desc) above 8 MiB, i.e.
 * roughly 64 B per tube plus 0.5 B per node), LBM_EDEVICE, LBM_ELAUNCH. */
lbm_status lbm_batch_step_noalloc(const lbm_batch_desc *desc, void *hip_stream);

/* Release the HIP graph lbm_batch_step keeps for this descriptor on the
 * current device (the library records one per distinct descriptor and device,
 * at most 16, and otherwise keeps them until the process ends).  Call it
 * before freeing the descriptor's buffers.  A later lbm_batch_step with the
 * same descriptor records a new graph.  Errors: LBM_EINVAL, LBM_EDEVICE. */
lbm_status lbm_batch_release(const lbm_batch_desc *desc);

/* Packed FP64 fields rho[total], u[total], T[total] of the state in f[0], g[0];
 * any may be NULL. */
lbm_status lbm_batch_moments(const lbm_batch_desc *desc, double *rho, double *u, double *T,
                             void *hip_stream);


/* ------------------------------------------------------------------------ */
/* Learned surrogate of the batched tubes: a 1-D neural operator that maps   */
/* (rho, u, T, gamma) of a tube to (rho, u, T) k = 16 lattice steps later.   */
/* The plain scheme above generates its training data, is the reference its */
/* error is measured against, and replaces it wherever a conservation or    */
/* admissibility check fails.  The paper has no learned component; only the */
/* fallback and the error reference are its method.                         */
/*                                                                          */
/* Network (tokens = patches of 4 nodes, C = 64 channels, 4 blocks):         */
/*   X  [M][16]  features (rho-0.5)/0.5, u/0.5, (T-1)/0.5, (gamma-1.4)/0.3   */
/*               of the 4 nodes of a patch, feature p*4 + c                  */
/*   H0 = X We^T + be                                       We [64][16]      */
/*   block b: Hc = H + bc + dwconv5(H)   (per channel, zero padding, taps    */
/*                                       kc[64][5] at token offsets -2..2)   */
/*            H' = Hc + W2 gelu(W1 Hc + b1) + b2    W1 [128][64], W2 [64][128] */
/*   Y  = H4 Wh^T + bh                                      Wh [12][64]      */
/*   out_c(node 4t+p) = in_c(node 4t+p) + 0.1 * Y[t][p*3 + c]               */
/* gelu(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).                  */
/* Matrix products take BF16 operands (weights and activations rounded to    */
/* nearest-even) on MFMA with FP32 accumulation; everything else is FP32.    */
/* Parameter vector (FP32, this order, LBM_SUR_NPARAMS = 69708 values):      */
/*   We, be, {kc, bc, W1, b1, W2, b2} x 4 blocks, Wh, bh  (row-major)        */
/* ------------------------------------------------------------------------ */
#define LBM_SUR_NPARAMS 69708
#define LBM_SUR_K 16 /* lattice steps per surrogate call */

typedef struct {
    int32_t abi_version;
    int32_t batch;        /* B tubes */
    int32_t length;       /* L nodes per tube, a multiple of 128 */
    const float *params;  /* device [LBM_SUR_NPARAMS] FP32 master parameters */
    void *params_bf16;    /* device, lbm_sur_bf16_bytes(): BF16 copies of the
                             weight matrices and their transposes, written by
                             lbm_sur_pack / lbm_sur_adam */
    void *workspace;      /* device, lbm_sur_workspace_bytes() bytes */
} lbm_sur_desc;

size_t lbm_sur_bf16_bytes(void);
size_t lbm_sur_workspace_bytes(const lbm_sur_desc *desc);

/* Refresh params_bf16 from params (after initialising or loading them). */
lbm_status lbm_sur_pack(const lbm_sur_desc *desc, void *hip_stream);

/* Inference: x [3][B][L] FP64 fields (rho, u, T), gamma [B] FP64 ->
 * y [3][B][L] FP64 predicted fields LBM_SUR_K steps later.  y may not
 * alias x.  active: NULL, or device int32 [B]: tubes with active[b] == 0
 * are skipped (their rows of y are not written). */
lbm_status lbm_sur_forward(const lbm_sur_desc *desc, const double *x, const double *gamma,
                           const int32_t *active, double *y, void *hip_stream);

/* Training step: forward on x, loss = mean over nodes and channels of
 * (Y_c - (target_c - x_c) / 0.1)^2, backward.  grads [LBM_SUR_NPARAMS] FP32
 * are overwritten; loss [1] FP32 (device). */
lbm_status lbm_sur_backward(const lbm_sur_desc *desc, const double *x, const double *gamma,
                            const double *target, float *grads, float *loss, void *hip_stream);

/* Adam on the FP32 master parameters (m, v: FP32 moments of the same size),
 * step >= 1, then refresh params_bf16.  Decoupled from the loss scale. */
lbm_status lbm_sur_adam(const lbm_sur_desc *desc, float *params, float *m, float *v,
                        const float *grads, float lr, float beta1, float beta2, float eps,
                        int64_t step, void *hip_stream);

/* Admission check of a surrogate step for every tube b: with n_b from
 * gamma_b (n = 2/(gamma-1) - 1), the change from x to y of the totals
 * mass = sum rho, momentum = sum rho u and energy = sum rho (u^2/2 +
 * (1+n) T/2) must equal what crosses the tube's open ends in LBM_SUR_K
 * steps (the balance laws of Sec. II: (K/r) times the difference of the
 * equilibrium fluxes rho u, rho (u^2 + T), rho u (u^2/2 + (3+n) T/2) at the
 * first and last node, end states averaged over x and y) within tol_mass,
 * tol_mom (relative to mass * sqrt(max T of x)) and tol_energy (relative);
 * y must be finite with rho > 0 and T > 0 at every node, and, if max_mach
 * > 0, |u| <= max_mach sqrt(T) at every node (the fourth-order D1Q7
 * equilibrium of Sec. IV stays positive up to |u| ~ 0.91 sqrt(T)).
 * accept[b] = 1 or 0 (device int32).  The totals use FP64 and a fixed
 * reduction order.  Errors: LBM_EINVAL, LBM_ELAUNCH. */
lbm_status lbm_sur_check(const lbm_sur_desc *desc, const double *x, const double *y,
                         const double *gamma, double tol_mass, double tol_mom, double tol_energy,
                         double max_mach, int32_t *accept, void *hip_stream);

/* Fallback preparation into the batch that runs the plain scheme for the
 * rejected tubes: `batch` must describe FP32 populations of exactly
 * desc->batch tubes of desc->length nodes (tube b owns nodes b*L ..
 * (b+1)*L-1), else LBM_EINVAL (size and type are checked on the host; a tube
 * whose device offsets differ gets nothing written and 0 steps).  For every
 * tube b with accept[b] == 0 and valid[b] == 0 the equilibrium populations
 * of x (f = f^eq, g = g^eq, Sec. IV) are written into batch->f[0],
 * batch->g[0] at the tube's slot.  valid[b] != 0 means those buffers already
 * hold the tube's populations at the time of x (it ran the plain scheme up
 * to that time), so the non-equilibrium part is kept.  batch->nsteps[b] =
 * steps (>= 0; LBM_SUR_K for one call) for every rejected tube (lift
 * writes it); accepted tubes' entries are left as they are, so a caller
 * that collects rejections over several calls zeroes nsteps first.
 * Errors: LBM_EINVAL, LBM_ELAUNCH. */
lbm_status lbm_sur_lift(const lbm_sur_desc *desc, const double *x, const int32_t *accept,
                        const int32_t *valid, const lbm_batch_desc *batch, int64_t steps,
                        void *hip_stream);

/* out[c][b][l] = accept[b] ? y : z (FP64 [3][B][L]); out may alias y or z.
 * valid[b] = accept[b] ? 0 : 1 (the batch buffers hold tube b's populations
 * at the new time exactly when it ran the plain scheme). */
lbm_status lbm_sur_merge(const lbm_sur_desc *desc, const int32_t *accept, const double *y,
                         const double *z, double *out, int32_t *valid, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
