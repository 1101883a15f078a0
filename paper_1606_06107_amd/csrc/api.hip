// C-ABI host library (declarations and contracts in include/lbm.h):
// argument validation, kernel launches on the caller's stream, HIP-graph
// capture and replay of multi-step calls, error strings.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "fd.hpp"
#include "launch.hpp"
#include "lbm.h"
#include "lbm_device.hpp"

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

lbm_status hip_fail(hipError_t e, const char *what) {
    return fail(LBM_ELAUNCH, "%s: %s", what, hipGetErrorString(e));
}

// The library targets gfx950 (MI355X) only.
lbm_status check_device() {
    int dev = 0, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(LBM_EDEVICE, "no HIP device available");
    if (hipGetDevice(&dev) != hipSuccess) return fail(LBM_EDEVICE, "hipGetDevice failed");
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess)
        return fail(LBM_EDEVICE, "hipGetDeviceProperties failed");
    if (strncmp(p.gcnArchName, "gfx950", 6) != 0)
        return fail(LBM_EDEVICE, "device %d is %s; this library is built for gfx950", dev,
                    p.gcnArchName);
    return LBM_OK;
}

int q_of(int lattice) {
    return lattice == LBM_D1Q7 ? 7 : lattice == LBM_D2Q49 ? 49 : lattice == LBM_D2Q37 ? 37 : 343;
}
int kind_of(int lattice) { return lattice == LBM_D2Q37 ? lbmx::kD2Q37 : lbmx::kTensor; }
size_t pop_bytes(int dtype) { return dtype == LBM_F32 ? 4 : 8; }

void default_tile(int dim, int tile[3]) {
    tile[2] = 1;
    if (dim == 1) { tile[0] = 256; tile[1] = 1; }
    else if (dim == 2) { tile[0] = 256; tile[1] = 1; }
    else { tile[0] = 64; tile[1] = 1; }
}

// Largest number of per-tile partial rows any supported launch can produce.
int64_t max_partial_rows(const lbm_desc *d) {
    const int64_t N = d->n[0] * d->n[1] * d->n[2];
    int64_t rows = (N + 255) / 256;  // field kernel
    static const int cand[][2] = {{64, 1}, {128, 1}, {256, 1}, {512, 1}, {1024, 1}, {64, 4},
                                  {32, 8}, {128, 2}, {64, 8}, {32, 16}, {16, 16}, {64, 2},
                                  {32, 2}, {16, 4}};
    for (auto &c : cand) {
        const int t[3] = {c[0], c[1], 1};
        int a, b, e;
        if (d->dim == 1 && c[1] != 1) continue;
        const int64_t n = lbmx::step_ntiles(d->dim, t, (int)d->n[0], (int)d->n[1], (int)d->n[2],
                                            &a, &b, &e);
        if (n > rows) rows = n;
    }
    return rows;
}

// Byte offset of the conservation monitor's row counter (one int64) in the
// workspace, after the partial rows.
size_t monitor_slot_offset(const lbm_desc *d) {
    const size_t rows = (size_t)max_partial_rows(d);
    return ((rows * (2 + d->dim) * sizeof(double) + 255) / 256) * 256;
}

// Sub-stepped rotational advection (g_substeps > 1): 17 N population values
// of scratch after the counter.
size_t substep_offset(const lbm_desc *d) { return monitor_slot_offset(d) + 256; }
size_t substep_bytes(const lbm_desc *d) {
    if (d->g_substeps <= 1) return 0;
    const size_t N = (size_t)(d->n[0] * d->n[1] * d->n[2]);
    return ((17 * N * (d->dtype == LBM_F32 ? 4 : 8) + 255) / 256) * 256;
}

lbm_status validate(const lbm_desc *d) {
    if (!d) return fail(LBM_EINVAL, "descriptor is NULL");
    if (d->abi_version != LBM_ABI_VERSION)
        return fail(LBM_EINVAL, "abi_version %d != %d", d->abi_version, LBM_ABI_VERSION);
    if (d->dim < 1 || d->dim > 3) return fail(LBM_EINVAL, "dim must be 1, 2 or 3");
    const int want = d->dim == 1 ? LBM_D1Q7 : d->dim == 2 ? LBM_D2Q49 : LBM_D3Q343;
    if (d->lattice != want && !(d->dim == 2 && d->lattice == LBM_D2Q37))
        return fail(LBM_EINVAL, "lattice %d does not match dim %d", d->lattice, d->dim);
    if (d->dtype != LBM_F32 && d->dtype != LBM_F64) return fail(LBM_EINVAL, "dtype must be F32 or F64");
    int64_t N = 1;
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1) return fail(LBM_EINVAL, "n[%d] = %lld < 1", a, (long long)d->n[a]);
        if (a >= d->dim && d->n[a] != 1) return fail(LBM_EINVAL, "unused axis %d must have n = 1", a);
        if (a < d->dim && d->bc[a] != LBM_BC_PERIODIC && d->bc[a] != LBM_BC_OPEN)
            return fail(LBM_EINVAL, "bc[%d] invalid", a);
        if (a < d->dim && d->bc[a] == LBM_BC_PERIODIC && d->n[a] < 3)
            return fail(LBM_EINVAL, "periodic axis %d needs n >= 3", a);
        if (d->n[a] > (1LL << 30)) return fail(LBM_EINVAL, "n[%d] too large", a);
        N *= d->n[a];
        if (N >= (1LL << 31)) return fail(LBM_EINVAL, "N must be < 2^31");
    }
    if ((uint64_t)N * (d->dtype == LBM_F32 ? 4u : 8u) >= (1ULL << 32))
        return fail(LBM_EINVAL, "N * sizeof(population) must be < 2^32 bytes per population");
    if (!(d->n_rot >= 0.0) || !isfinite(d->n_rot)) return fail(LBM_EINVAL, "n_rot must be >= 0");
    if (!(d->tau > 0.5) || !isfinite(d->tau)) return fail(LBM_EINVAL, "tau must be > 0.5");
    if (d->g_substeps < 0 || d->g_substeps > 64) return fail(LBM_EINVAL, "g_substeps must be in [0, 64]");
    if (!d->f[0] || !d->f[1] || !d->g[0] || !d->g[1])
        return fail(LBM_EINVAL, "population buffers must not be NULL");
    if (d->f[0] == d->f[1] || d->g[0] == d->g[1] || d->f[0] == d->g[0] || d->f[1] == d->g[1])
        return fail(LBM_EINVAL, "population buffers must be distinct");
    if (!d->workspace) return fail(LBM_EINVAL, "workspace must not be NULL");
    if (((uintptr_t)d->workspace) % 256) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    return LBM_OK;
}

}  // namespace

namespace lbmx {
void set_error(const char *msg) { g_err = msg; }
}  // namespace lbmx

struct lbm_sim_s {
    lbm_desc d;
    hipStream_t stream;    // caller's stream
    hipStream_t capture;   // private stream used only to record graphs
    int fcur = 0, gcur = 0;               // buffer indices of the current f and g
    int layout = lbmx::kLayoutStreamed;   // what f[fcur] holds (just initialised)
    int inplace = 0;                      // translational streaming in one buffer
    int blocked = 0;                      // value order of f (lbmx::pop_index)
    double fd = 0.0;                      // > 0: finite-difference update, this Courant factor
    int64_t t = 0;
    int tile[3];
    int graphs = 1;
    int64_t mon_every = 0;
    double *mon_series = nullptr;
    int64_t mon_cap = 0;
    int debug = 0;                        // lbm_set_debug flags
    struct Entry {
        int64_t n, t0, every, cap;
        int fcur, gcur, layout, inplace, tile0, tile1, debug;
        double *series;
        hipGraphExec_t exec;
    };
    std::vector<Entry> cache;
    // recorded on `stream` after every graph launch: a graph is destroyed
    // only once its last launch (all run in stream order) has finished
    hipEvent_t launched = nullptr;
};

namespace {

// Wait for the handle's last graph launch before a graph is destroyed.
void wait_launched(lbm_sim s) {
    if (s->launched) hipEventSynchronize(s->launched);
}

void clear_cache(lbm_sim s) {
    if (!s->cache.empty()) wait_launched(s);
    for (auto &e : s->cache) hipGraphExecDestroy(e.exec);
    s->cache.clear();
}

int64_t N_of(const lbm_desc &d) { return d.n[0] * d.n[1] * d.n[2]; }

int64_t *monitor_slot(lbm_sim s) {
    return reinterpret_cast<int64_t *>(static_cast<char *>(s->d.workspace) + monitor_slot_offset(&s->d));
}

// Host-side state after n more steps (the time counter aside).
void advance(lbm_sim s, int64_t n) {
    if (n <= 0) return;
    s->gcur = (int)((s->gcur + n) & 1);
    if (s->fd > 0.0) {  // values stay at their nodes
        s->fcur = (int)((s->fcur + n) & 1);
        s->layout = lbmx::kLayoutStreamed;
    } else if (s->inplace) {
        // even steps turn kLayoutStreamed into kLayoutSwapped, odd steps back
        if (n & 1)
            s->layout = s->layout == lbmx::kLayoutStreamed ? lbmx::kLayoutSwapped : lbmx::kLayoutStreamed;
    } else {
        s->fcur = (int)((s->fcur + n) & 1);
        s->layout = lbmx::kLayoutPost;
    }
}

// Enqueue one finite-difference time step (lbm_set_fd).
hipError_t enqueue_step_fd(lbm_sim s, hipStream_t st) {
    const lbm_desc &d = s->d;
    lbmx::FdArgs a;
    a.f_in = d.f[s->fcur];
    a.g_in = d.g[s->gcur];
    a.f_out = d.f[s->fcur ^ 1];
    a.g_out = d.g[s->gcur ^ 1];
    a.n0 = (int)d.n[0];
    a.n1 = (int)d.n[1];
    a.open0 = d.bc[0] == LBM_BC_OPEN;
    a.open1 = d.dim >= 2 && d.bc[1] == LBM_BC_OPEN;
    a.N = (uint32_t)N_of(d);
    a.lambda = s->fd;
    a.omega = s->fd / d.tau;
    a.n_rot = d.n_rot;
    int tx, ty;
    lbmx::fd_tile(d.dim, &tx, &ty);
    a.tiles0 = (a.n0 + tx - 1) / tx;
    a.ntiles = a.tiles0 * (d.dim >= 2 ? (a.n1 + ty - 1) / ty : 1);
    hipError_t e = lbmx::launch_step_fd(d.dtype, d.dim, kind_of(d.lattice), a, st);
    if (e != hipSuccess) return e;
    advance(s, 1);
    s->t += 1;
    return hipSuccess;
}

lbmx::FieldArgs field_args(lbm_sim s);

// Enqueue one time step with the rotational advection in sub-steps.
hipError_t enqueue_step_sub(lbm_sim s, hipStream_t st) {
    const lbm_desc &d = s->d;
    const lbmx::FieldArgs a = field_args(s);
    if (s->mon_every > 0 && s->t % s->mon_every == 0) {  // totals of time t
        lbmx::FieldArgs fa = a;
        fa.partials = (double *)d.workspace;
        int nb = 0;
        hipError_t e = lbmx::launch_fields(d.dtype, d.dim, kind_of(d.lattice), fa, &nb, st);
        if (e == hipSuccess)
            e = lbmx::launch_reduce_series((const double *)d.workspace, nb, 2 + d.dim, s->mon_series, s->mon_cap,
                                           monitor_slot(s), st);
        if (e != hipSuccess) return e;
    }
    void *scratch = static_cast<char *>(d.workspace) + substep_offset(&d);
    hipError_t e = lbmx::launch_step_sub(d.dtype, d.dim, kind_of(d.lattice), a, d.f[s->fcur ^ 1], d.g[s->gcur ^ 1],
                                         scratch, d.g_substeps, 1.0 / d.tau, st);
    if (e != hipSuccess) return e;
    advance(s, 1);
    s->t += 1;
    return hipSuccess;
}

// Debug poisoning (LBM_DEBUG_POISON): quiet NaN into the buffers the next
// step writes without reading (the ping-pong destinations), so a value the
// step fails to write shows up as NaN.
hipError_t poison_destinations(lbm_sim s, hipStream_t st) {
    const lbm_desc &d = s->d;
    const size_t N = (size_t)N_of(d);
    hipError_t e = lbmx::launch_fill_nan(d.dtype, d.g[s->gcur ^ 1], 7 * N, st);
    if (e == hipSuccess && !s->inplace) e = lbmx::launch_fill_nan(d.dtype, d.f[s->fcur ^ 1], (size_t)q_of(d.lattice) * N, st);
    return e;
}

// Enqueue one time step on stream st and advance the host-side state.
hipError_t enqueue_step(lbm_sim s, hipStream_t st) {
    if (s->debug & LBM_DEBUG_POISON) {
        const hipError_t e = poison_destinations(s, st);
        if (e != hipSuccess) return e;
    }
    if (s->fd > 0.0) return enqueue_step_fd(s, st);
    if (s->d.g_substeps > 1) return enqueue_step_sub(s, st);
    const lbm_desc &d = s->d;
    lbmx::StepArgs a;
    a.f_in = d.f[s->fcur];
    a.g_in = d.g[s->gcur];
    a.f_out = s->inplace ? d.f[s->fcur] : d.f[s->fcur ^ 1];
    a.g_out = d.g[s->gcur ^ 1];
    a.n0 = (int)d.n[0];
    a.n1 = (int)d.n[1];
    a.n2 = (int)d.n[2];
    a.open0 = d.dim >= 1 && d.bc[0] == LBM_BC_OPEN;
    a.open1 = d.dim >= 2 && d.bc[1] == LBM_BC_OPEN;
    a.open2 = d.dim >= 3 && d.bc[2] == LBM_BC_OPEN;
    a.N = (uint32_t)N_of(d);
    a.layout = s->layout;
    a.blocked = s->blocked;
    a.scheme = !s->inplace ? lbmx::kSchemePingPong
                           : (s->layout == lbmx::kLayoutStreamed ? lbmx::kSchemeInPlaceEven
                                                                 : lbmx::kSchemeInPlaceOdd);
    a.omega = 1.0 / d.tau;
    a.n_rot = d.n_rot;
    a.ntiles = lbmx::step_ntiles(d.dim, s->tile, a.n0, a.n1, a.n2, &a.tiles0, &a.tiles1, &a.tiles2);
    // Tile order alternates from step to step (odd in-place steps; every
    // other ping-pong step, by buffer parity), a function of state that the
    // graph cache keys on (layout, fcur).
    a.reverse = s->inplace ? (a.scheme == lbmx::kSchemeInPlaceOdd ? 1 : 0) : s->fcur;
    // Monitored steps depend on t mod every only; the row they fill comes
    // from the device-side counter (set by lbm_set_monitor), so a recorded
    // graph of steps replays correctly from any start with the same phase.
    const bool mon = s->mon_every > 0 && s->t % s->mon_every == 0;
    a.partials = mon ? (double *)d.workspace : nullptr;
    hipError_t e = lbmx::launch_step(d.dtype, d.dim, kind_of(d.lattice), s->tile, a, st);
    if (e != hipSuccess) return e;
    if (mon) {
        e = lbmx::launch_reduce_series((const double *)d.workspace, a.ntiles, 2 + d.dim, s->mon_series,
                                       s->mon_cap, monitor_slot(s), st);
        if (e != hipSuccess) return e;
    }
    advance(s, 1);
    s->t += 1;
    return hipSuccess;
}

// In-place streaming needs a bijective scatter x -> x + c: every axis
// periodic; 1-D and 2-D lattices.
bool inplace_possible(const lbm_desc &d) {
    if (d.dim > 2) return false;
    for (int a = 0; a < d.dim; ++a)
        if (d.bc[a] != LBM_BC_PERIODIC) return false;
    return true;
}

// The blocked order puts one 64-node tile's populations in one block: 3-D
// grids whose rows are whole blocks.
bool blocked_possible(const lbm_desc &d) { return d.dim == 3 && d.n[0] % lbmx::kBlk == 0; }

// Field/export arguments for the current state.
lbmx::FieldArgs field_args(lbm_sim s) {
    const lbm_desc &d = s->d;
    lbmx::FieldArgs a = {};
    a.f = d.f[s->fcur];
    a.g = d.g[s->gcur];
    a.n0 = (int)d.n[0];
    a.n1 = (int)d.n[1];
    a.n2 = (int)d.n[2];
    a.open0 = d.bc[0] == LBM_BC_OPEN;
    a.open1 = d.dim >= 2 && d.bc[1] == LBM_BC_OPEN;
    a.open2 = d.dim >= 3 && d.bc[2] == LBM_BC_OPEN;
    a.N = (uint32_t)N_of(d);
    a.layout = s->layout;
    a.blocked = s->blocked;
    a.n_rot = d.n_rot;
    return a;
}

lbm_status make_sim(const lbm_desc *desc, void *stream, lbm_sim *out) {
    lbm_status st = validate(desc);
    if (st) return st;
    if (!out) return fail(LBM_EINVAL, "out handle pointer is NULL");
    st = check_device();
    if (st) return st;
    lbm_sim s = new (std::nothrow) lbm_sim_s();
    if (!s) return fail(LBM_ENOMEM, "out of host memory");
    s->d = *desc;
    s->stream = (hipStream_t)stream;
    default_tile(desc->dim, s->tile);
    s->inplace = inplace_possible(*desc) && desc->g_substeps <= 1 ? 1 : 0;
    s->blocked = blocked_possible(*desc) ? 1 : 0;
    if (hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return fail(LBM_EDEVICE, "hipStreamCreateWithFlags failed");
    }
    *out = s;
    return LBM_OK;
}

// The instantiated graph of nsteps launches from the current state: from the
// cache, or recorded on the private stream and instantiated (and cached).
// The key holds everything the recorded launches depend on: buffer indices,
// layout, scheme, tile, monitor settings and the phase t mod every.
lbm_status graph_for(lbm_sim s, int64_t nsteps, hipGraphExec_t *out) {
    const bool mon = s->mon_every > 0;
    const int64_t t0key = mon ? s->t % s->mon_every : -1;
    for (auto &en : s->cache) {
        if (en.n == nsteps && en.fcur == s->fcur && en.gcur == s->gcur && en.layout == s->layout &&
            en.inplace == s->inplace && en.t0 == t0key && en.tile0 == s->tile[0] &&
            en.tile1 == s->tile[1] && en.every == s->mon_every && en.cap == s->mon_cap &&
            en.series == s->mon_series && en.debug == s->debug) {
            *out = en.exec;
            return LBM_OK;
        }
    }
    const int fcur0 = s->fcur, gcur0 = s->gcur, lay0 = s->layout;
    const int64_t t0 = s->t;
    hipError_t e = hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) e = enqueue_step(s, s->capture);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s->capture, &graph);
    s->fcur = fcur0;  // recording only: the host-side state stays where it was
    s->gcur = gcur0;
    s->layout = lay0;
    s->t = t0;
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        return hip_fail(e != hipSuccess ? e : e2, "graph capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    if (s->cache.size() >= 8) {
        wait_launched(s);
        hipGraphExecDestroy(s->cache.front().exec);
        s->cache.erase(s->cache.begin());
    }
    s->cache.push_back({nsteps, t0key, s->mon_every, s->mon_cap, fcur0, gcur0, lay0, s->inplace,
                        s->tile[0], s->tile[1], s->debug, s->mon_series, exec});
    *out = exec;
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_desc *desc) {
    if (!desc || desc->dim < 1 || desc->dim > 3) return 0;
    for (int a = 0; a < 3; ++a)
        if (desc->n[a] < 1) return 0;
    return substep_offset(desc) + substep_bytes(desc);
}

lbm_status lbm_init(const lbm_desc *desc, const double *rho, const double *u, const double *T,
                    void *hip_stream, lbm_sim *out) {
    if (!rho || !u || !T) return fail(LBM_EINVAL, "rho, u and T must not be NULL");
    lbm_sim s = nullptr;
    lbm_status st = make_sim(desc, hip_stream, &s);
    if (st) return st;
    lbmx::InitArgs a{rho, u, T, desc->f[0], desc->g[0], (uint32_t)N_of(*desc), s->blocked};
    hipError_t e = lbmx::launch_init(desc->dtype, desc->dim, kind_of(desc->lattice), a, s->stream);
    if (e != hipSuccess) {
        lbm_destroy(s);
        return hip_fail(e, "init launch");
    }
    *out = s;
    return LBM_OK;
}

lbm_status lbm_init_populations(const lbm_desc *desc, const void *f0, const void *g0,
                                void *hip_stream, lbm_sim *out) {
    if (!f0 || !g0) return fail(LBM_EINVAL, "f0 and g0 must not be NULL");
    lbm_sim s = nullptr;
    lbm_status st = make_sim(desc, hip_stream, &s);
    if (st) return st;
    const size_t N = (size_t)N_of(*desc), b = pop_bytes(desc->dtype);
    hipError_t e = hipSuccess;
    if (s->blocked) {  // reorder into f[0], or into f[1] when f0 is f[0]
        s->fcur = f0 == desc->f[0] ? 1 : 0;
        e = lbmx::launch_to_blocked(desc->dtype, q_of(desc->lattice), (uint32_t)N, f0, desc->f[s->fcur],
                                    s->stream);
    } else if (f0 != desc->f[0]) {
        e = hipMemcpyAsync(desc->f[0], f0, (size_t)q_of(desc->lattice) * N * b,
                           hipMemcpyDeviceToDevice, s->stream);
    }
    if (e == hipSuccess && g0 != desc->g[0])
        e = hipMemcpyAsync(desc->g[0], g0, 7 * N * b, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) {
        lbm_destroy(s);
        return hip_fail(e, "population copy");
    }
    *out = s;
    return LBM_OK;
}

lbm_status lbm_step(lbm_sim s, int64_t nsteps) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return LBM_OK;
    if (s->fd > 0.0 && s->mon_every > 0)
        return fail(LBM_EUNSUPPORTED, "the conservation monitor is not available with the finite-difference update");
    if (!s->graphs || nsteps == 1) {
        for (int64_t k = 0; k < nsteps; ++k) {
            hipError_t e = enqueue_step(s, s->stream);
            if (e != hipSuccess) return hip_fail(e, "step launch");
        }
        return LBM_OK;
    }
    hipGraphExec_t exec = nullptr;
    lbm_status st = graph_for(s, nsteps, &exec);
    if (st) return st;
    hipError_t e = hipGraphLaunch(exec, s->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    if (!s->launched && hipEventCreateWithFlags(&s->launched, hipEventDisableTiming) != hipSuccess)
        s->launched = nullptr;
    if (s->launched) hipEventRecord(s->launched, s->stream);
    advance(s, nsteps);
    s->t += nsteps;
    return LBM_OK;
}

lbm_status lbm_prepare(lbm_sim s, int64_t nsteps) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (!s->graphs || nsteps <= 1) return LBM_OK;
    if (s->fd > 0.0 && s->mon_every > 0)
        return fail(LBM_EUNSUPPORTED, "the conservation monitor is not available with the finite-difference update");
    hipGraphExec_t exec = nullptr;
    return graph_for(s, nsteps, &exec);
}

lbm_status lbm_moments(lbm_sim s, double *rho, double *u, double *T, double *totals) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    const lbm_desc &d = s->d;
    lbmx::FieldArgs a = field_args(s);
    a.rho = rho;
    a.u = u;
    a.T = T;
    a.partials = totals ? (double *)d.workspace : nullptr;
    if (!rho && !u && !T && !totals) return LBM_OK;
    int nb = 0;
    hipError_t e = lbmx::launch_fields(d.dtype, d.dim, kind_of(d.lattice), a, &nb, s->stream);
    if (e != hipSuccess) return hip_fail(e, "moments launch");
    if (totals) {
        e = lbmx::launch_reduce((const double *)d.workspace, nb, 2 + d.dim, totals, s->stream);
        if (e != hipSuccess) return hip_fail(e, "reduce launch");
    }
    return LBM_OK;
}

lbm_status lbm_populations(lbm_sim s, void *f_out, void *g_out) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (!f_out && !g_out) return LBM_OK;
    const lbm_desc &d = s->d;
    for (int k = 0; k < 2; ++k)
        if ((f_out && (f_out == d.f[k] || f_out == d.g[k])) ||
            (g_out && (g_out == d.f[k] || g_out == d.g[k])))
            return fail(LBM_EINVAL, "export buffers must differ from the state buffers");
    lbmx::FieldArgs a = field_args(s);
    a.f_out = f_out;
    a.g_out = g_out;
    hipError_t e = lbmx::launch_export(d.dtype, d.dim, kind_of(d.lattice), a, s->stream);
    if (e != hipSuccess) return hip_fail(e, "export launch");
    return LBM_OK;
}

lbm_status lbm_set_monitor(lbm_sim s, int64_t every, double *series, int64_t capacity) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (every < 0 || capacity < 0) return fail(LBM_EINVAL, "every and capacity must be >= 0");
    if (every > 0 && (!series || capacity == 0))
        return fail(LBM_EINVAL, "series buffer and capacity required when every > 0");
    if (every > 0) {  // the next recorded time t = k * every >= now fills row k
        const hipError_t e = lbmx::launch_set_i64(monitor_slot(s), (s->t + every - 1) / every, s->stream);
        if (e != hipSuccess) return hip_fail(e, "monitor counter");
    }
    s->mon_every = every;
    s->mon_series = every > 0 ? series : nullptr;
    s->mon_cap = every > 0 ? capacity : 0;
    return LBM_OK;
}

lbm_status lbm_time(lbm_sim s, int64_t *t) {
    if (!s || !t) return fail(LBM_EINVAL, "NULL argument");
    *t = s->t;
    return LBM_OK;
}

lbm_status lbm_set_debug(lbm_sim s, int32_t flags) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (flags & ~LBM_DEBUG_POISON) return fail(LBM_EINVAL, "unknown debug flags 0x%x", flags);
    s->debug = flags;
    return LBM_OK;
}

lbm_status lbm_set_graphs(lbm_sim s, int32_t enable) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    s->graphs = enable ? 1 : 0;
    return LBM_OK;
}

lbm_status lbm_set_inplace(lbm_sim s, int32_t enable) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (s->t != 0 || s->layout != lbmx::kLayoutStreamed)
        return fail(LBM_EINVAL, "the streaming scheme can only be chosen before the first step");
    if (enable && !inplace_possible(s->d))
        return fail(LBM_EUNSUPPORTED, "in-place streaming needs a 1-D or 2-D grid periodic in every axis");
    if (enable && s->d.g_substeps > 1)
        return fail(LBM_EUNSUPPORTED, "the sub-stepped rotational advection ping-pongs");
    if (enable && s->fd > 0.0)
        return fail(LBM_EUNSUPPORTED, "the finite-difference update ping-pongs");
    s->inplace = enable ? 1 : 0;
    clear_cache(s);
    return LBM_OK;
}

lbm_status lbm_set_fd(lbm_sim s, double courant) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (s->t != 0 || s->layout != lbmx::kLayoutStreamed)
        return fail(LBM_EINVAL, "the update can only be chosen before the first step");
    if (!(courant >= 0.0 && courant <= 1.0)) return fail(LBM_EINVAL, "courant must be in [0, 1]");
    if (courant > 0.0 && s->d.dim > 2)
        return fail(LBM_EUNSUPPORTED, "the finite-difference update runs on 1-D and 2-D grids");
    if (courant > 0.0 && s->d.g_substeps > 1)
        return fail(LBM_EUNSUPPORTED, "the finite-difference update has no sub-stepped rotational advection");
    s->fd = courant;
    if (courant > 0.0) s->inplace = 0;
    else s->inplace = inplace_possible(s->d) && s->d.g_substeps <= 1 ? 1 : 0;
    clear_cache(s);
    return LBM_OK;
}

lbm_status lbm_set_blocked(lbm_sim s, int32_t enable) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (s->t != 0 || s->layout != lbmx::kLayoutStreamed)
        return fail(LBM_EINVAL, "the population order can only be chosen before the first step");
    enable = enable ? 1 : 0;
    if (enable && !blocked_possible(s->d))
        return fail(LBM_EUNSUPPORTED, "the blocked order needs a 3-D grid with n0 a multiple of %d", lbmx::kBlk);
    if (enable == s->blocked) return LBM_OK;
    const lbm_desc &d = s->d;
    const int src = s->fcur, dst = s->fcur ^ 1;
    hipError_t e;
    if (enable) {
        e = lbmx::launch_to_blocked(d.dtype, q_of(d.lattice), (uint32_t)N_of(d), d.f[src], d.f[dst], s->stream);
    } else {
        lbmx::FieldArgs a = field_args(s);
        a.f_out = d.f[dst];
        e = lbmx::launch_export(d.dtype, d.dim, kind_of(d.lattice), a, s->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "reorder launch");
    s->fcur = dst;
    s->blocked = enable;
    if (enable) {
        s->tile[0] = lbmx::kBlk;
        s->tile[1] = s->tile[2] = 1;
    }
    clear_cache(s);
    return LBM_OK;
}

lbm_status lbm_set_tile(lbm_sim s, int32_t tx, int32_t ty, int32_t tz) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    const int t[3] = {tx, ty, tz};
    if (!lbmx::step_tile_supported(s->d.dtype, s->d.dim, kind_of(s->d.lattice), t))
        return fail(LBM_EUNSUPPORTED, "tile %dx%dx%d not compiled for dim %d", tx, ty, tz, s->d.dim);
    if (s->blocked && (tx != lbmx::kBlk || ty != 1 || tz != 1))
        return fail(LBM_EUNSUPPORTED, "the blocked population order runs with tile %dx1x1 only", lbmx::kBlk);
    s->tile[0] = tx;
    s->tile[1] = ty;
    s->tile[2] = tz;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_sim s) {
    if (!s) return LBM_OK;
    clear_cache(s);
    if (s->capture) hipStreamDestroy(s->capture);
    if (s->launched) hipEventDestroy(s->launched);
    delete s;
    return LBM_OK;
}

const char *lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_lattice_info(int32_t lattice, int32_t *Q, double *r, double *w, int32_t *c) {
    if (lattice != LBM_D1Q7 && lattice != LBM_D2Q49 && lattice != LBM_D3Q343 && lattice != LBM_D2Q37)
        return fail(LBM_EINVAL, "unknown lattice %d", lattice);
    const int q = q_of(lattice);
    const int D = lattice == LBM_D1Q7 ? 1 : (lattice == LBM_D2Q49 || lattice == LBM_D2Q37) ? 2 : 3;
    constexpr lbmx::DirTable<2, lbmx::kD2Q37> dirs37;
    if (Q) *Q = q;
    if (r) *r = lbmx::kR;
    for (int s = 0; s < q; ++s) {
        const int i = lattice == LBM_D2Q37 ? dirs37.v[s] : s;  // direction of storage slot s
        const int cx = lbmx::cx_of(i), cy = D >= 2 ? lbmx::cy_of(i) : 0, cz = D >= 3 ? lbmx::cz_of(i) : 0;
        if (w) {
            if (lattice == LBM_D2Q37) w[s] = lbmx::Lat<2, lbmx::kD2Q37>::w(i);
            else
                w[s] = lbmx::kW1[cx < 0 ? -cx : cx] * (D >= 2 ? lbmx::kW1[cy < 0 ? -cy : cy] : 1.0) *
                       (D >= 3 ? lbmx::kW1[cz < 0 ? -cz : cz] : 1.0);
        }
        if (c) {
            c[3 * s] = cx;
            c[3 * s + 1] = cy;
            c[3 * s + 2] = cz;
        }
    }
    return LBM_OK;
}

}  // extern "C"
