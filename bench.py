"""Benchmark of the decoupled Hermite lattice Boltzmann hot path on one GPU.

Workload (the metric's configuration): 2-D periodic compressible flow on
D2Q49 (translational) + D1Q7 (rotational), 1024 x 1024 nodes, FP32
populations with FP64 moments/temperature, gamma = 1.4 (n = 3), tau = 1,
seeded smooth random fields with Mach 0.3, conservation totals reduced in
FP64 every 100 steps (fused into the step).  One "step" = one time step of
the whole grid.  Inputs are resident in HBM before timing.

Prints ONE JSON line (rank 0).  --gpus N > 1 is not supported: the benchmark
runs on a single GPU.  Besides the headline workload the line carries
`extra` measurements of the other workloads (1-D tube, 3-D turbulence,
batched tubes, learned surrogate vs plain LBM); --no-extras skips them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s

# L2-to-memory bytes per step launch of the headline kernels (the even and
# odd in-place steps, averaged) from rocprofv3 FETCH_SIZE and WRITE_SIZE,
# scaled by the same counters on a plain device copy of known size
# (profiles/k_step_12_d2q49_1024x1024_fp32.md), per tile shape; valid only for
# the sources they were taken on (sha256 of the files below).
TRAFFIC = {"nodes": 1024 * 1024, "inplace": True,
           "bytes": {(16, 16): 522_077_399, (32, 8): 498_591_562, (32, 16): 476_071_477,
                     (64, 2): 491_743_786, (64, 4): 490_428_396, (64, 8): 475_393_660,
                     (128, 2): 490_100_131, (256, 1): 488_426_496},
           "sha256":
               "97c76ffa246e60889cfc500938e320a924fe0746d7ff286764ed118950a6605b"}
TRAFFIC_SOURCES = ("paper_1606_06107_amd/csrc/step_impl.hpp", "paper_1606_06107_amd/csrc/lbm_device.hpp",
                   "paper_1606_06107_amd/csrc/launch.hpp", "paper_1606_06107_amd/csrc/step_12_f32_inplace.hip",
                   "paper_1606_06107_amd/_build.py")


def kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


METRIC = "MLUPS & % HBM roofline; surrogate vs plain LBM speedup at <=1e-2 L1 error"


def _cpu_model():
    """Model name of the host CPU, with its family/model numbers (a virtual
    machine may report only a generic name)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k = k.strip()
                if k in ("model name", "cpu family", "model") and k not in info:
                    info[k] = v.strip()
                if len(info) == 3:
                    break
    except OSError:
        pass
    return f"{info.get('model name', 'unknown')} (family {info.get('cpu family', '?')}, model {info.get('model', '?')})"


def cpu_baseline(nx, ny, steps, threads, single=(512, 512, 30), parity_steps=50):
    """The CPU oracle (plain C, FP64) on bounded samples of the same workload:
    all of this process's host cores (at most `threads`), and one core.  The
    all-core run also gives the FP32 GPU path's error against the oracle on
    the benchmark grid: L-inf of rho, u, T after `parity_steps` steps."""
    import numpy as np
    import torch

    import oracle
    import workloads
    from paper_1606_06107_amd import Sim

    def run(nx_, ny_, steps_, th, snap=0):
        used = oracle.set_threads(th)
        w = workloads.Periodic2D(nx=nx_, ny=ny_)
        rho, u, T = w.fields()
        G = oracle.Grid(oracle.D2Q49, (nx_, ny_), n_rot=w.n_rot, tau=w.tau)
        f, g = G.init_eq(rho, u, T)
        G.step(f, g, 1)  # warm-up (page faults, thread start); step 1 of the trajectory
        done, dt, moments = 1, 0.0, None
        for seg in ([snap - 1, steps_ - snap + 1] if snap > 1 else [steps_]):
            t0 = time.perf_counter()
            G.step(f, g, seg)
            dt += time.perf_counter() - t0
            done += seg
            if done == snap:
                moments = G.moments(f, g)[:3]
        assert np.isfinite(f).all()
        return used, nx_ * ny_ * steps_ / dt / 1e6, dt, moments, w

    used, mlups, dt, orc, w = run(nx, ny, steps, threads, snap=parity_steps)
    sim = Sim((nx, ny), n_rot=w.n_rot, tau=w.tau, dtype=torch.float32).init(*w.fields())
    sim.step(parity_steps)
    gpu = [t.cpu().numpy() for t in sim.moments(totals=False)[:3]]
    del sim
    err = {k: float(np.abs(np.asarray(a) - np.asarray(b)).max()) for k, a, b in zip(("rho", "u", "T"), gpu, orc)}
    s_nx, s_ny, s_steps = single
    _, mlups1, dt1, _, _ = run(s_nx, s_ny, s_steps, 1)
    oracle.set_threads(threads)
    return {"value": round(mlups, 4), "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"{nx}x{ny} nodes x {steps} steps of the same 2-D workload, FP64, "
                      f"{used} threads, {dt:.1f} s wall",
            "single_core": {"value": round(mlups1, 4), "unit": "MLUPS",
                            "sample": f"{s_nx}x{s_ny} nodes x {s_steps} steps, 1 thread, {dt1:.1f} s wall"},
            "fp32_gpu_vs_oracle_linf": {"steps": parity_steps, **{k: float(f"{v:.3g}") for k, v in err.items()}},
            "cpu_model": _cpu_model(), "host_cpus_visible": len(os.sched_getaffinity(0))}


def copy_bandwidth(mbytes, reps=10):
    """Device-to-device copy of `mbytes` MB with the library's plain copy
    kernel (lbm_stream_copy), GB/s counting the bytes read plus the bytes
    written; median of `reps`.  Also torch's copy of the same buffers."""
    import ctypes

    import torch

    from paper_1606_06107_amd import _lib
    lib = _lib.load()
    n = int(mbytes * 1e6) // 16 * 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    out = {}
    for name, fn in (("lbm_stream_copy", lambda: _lib.check(lib.lbm_stream_copy(
            ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), n * 4,
            ctypes.c_void_p(stream.cuda_stream)))), ("torch", lambda: dst.copy_(src))):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        ts.sort()
        out[name] = round(2 * n * 4 / (ts[len(ts) // 2] * 1e-3) / 1e9, 1)
    assert bool(torch.equal(dst, src))
    del src, dst
    torch.cuda.empty_cache()
    return out


def _events(stream):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    return a, b


def extra_tube_1d():
    """The 1-D workloads, FP64, 1000 nodes x 1000 steps: the classic Sod tube
    (rotational advection in 4 sub-steps) and the Sec. VI tube's states with
    the update as written, each as one HIP graph of per-step kernels and as a
    batch of one (the whole time loop on chip in one launch)."""
    import numpy as np
    import torch

    import workloads
    from paper_1606_06107_amd import Batch, Sim

    def timed_sim(w):
        sim = Sim((w.N,), bc=["open"], n_rot=w.n_rot, tau=w.tau, dtype=torch.float64,
                  g_substeps=w.g_substeps).init(*w.fields())
        sim.step(w.steps)  # warm
        sim.init(*w.fields()).prepare(w.steps)  # a new handle: record its graph before timing
        a, b = _events(sim.stream)
        torch.cuda.synchronize()
        a.record(sim.stream)
        sim.step(w.steps)
        b.record(sim.stream)
        torch.cuda.synchronize()
        return sim, a.elapsed_time(b)

    def timed_batch(w):
        rho0, u0, T0_ = w.fields()
        bt = Batch([w.N], [w.n_rot], [w.tau], [w.steps], dtype=torch.float64, g_substeps=w.g_substeps)
        bt.init(rho0, np.asarray(u0).reshape(-1), T0_).step()  # capture + warm
        bt.init(rho0, np.asarray(u0).reshape(-1), T0_)
        a, b = _events(bt.stream)
        torch.cuda.synchronize()
        a.record(bt.stream)
        bt.step()
        b.record(bt.stream)
        torch.cuda.synchronize()
        return bt, a.elapsed_time(b)

    out = {}
    for name, w, what in (("classic_sod", workloads.tube_1d(),
                           "1-D classic Sod (1,0,1)|(0.125,0,0.1), 1000 nodes, n=4, tau=1, rotational advection "
                           "in 4 sub-steps, FP64, 1000 steps"),
                          ("paper_tube", workloads.paper_tube_1d(),
                           "1-D tube (4,0,4)|(1,0,1), 1000 nodes, n=4, tau=0.8, FP64, 1000 steps")):
        sim, ms = timed_sim(w)
        r1, u1, T1, _ = sim.moments()
        bt, ms_b = timed_batch(w)
        r2, u2, T2 = bt.moments()
        ok = bool(torch.isfinite(T1).all().item() and (r1.min() > 0).item() and (T1.min() > 0).item())
        diff = max(float((r1 - r2).abs().max()), float((u1.reshape(-1) - u2).abs().max()),
                   float((T1 - T2).abs().max()))
        out[name] = {"workload": what, "finite_positive": ok,
                     "per_step_kernels": {"ms_total": round(ms, 3), "us_per_step": round(1000 * ms / w.steps, 2),
                                          "MLUPS": round(w.N * w.steps / ms / 1e3, 1)},
                     "on_chip_batch_of_one": {"ms_total": round(ms_b, 3),
                                              "us_per_step": round(1000 * ms_b / w.steps, 3),
                                              "MLUPS": round(w.N * w.steps / ms_b / 1e3, 1),
                                              "max_abs_diff_vs_per_step": diff}}
        bt.release()
        del sim, bt
    return out


def extra_3d(steps=10):
    """256^3 decaying turbulence, D3Q343 + D1Q7 FP32, gamma = 1.4: the
    default blocked population order, and the plain [Q][N] order beside it."""
    import torch

    import workloads
    from paper_1606_06107_amd import Sim
    w = workloads.Turbulence3D()
    N = w.n ** 3

    def run(blocked):
        sim = Sim((w.n,) * 3, n_rot=w.n_rot, tau=w.tau, dtype=torch.float32).init(*w.fields())
        sim.set_blocked(blocked)
        sim.step(2)
        sim.prepare(steps)
        a, b = _events(sim.stream)
        torch.cuda.synchronize()
        a.record(sim.stream)
        sim.step(steps)
        b.record(sim.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        T = sim.moments(totals=False)[2]
        ok = bool(torch.isfinite(T).all().item())
        del sim, T
        torch.cuda.empty_cache()
        return ms, ok

    ms, ok = run(True)
    ms_plain, ok_plain = run(False)
    gbs = N * 2800 / (ms * 1e-3) / 1e9
    probe = pattern_probe_3d(w.n, steps)
    return {"workload": "3-D 256^3 turbulence, D3Q343+D1Q7 FP32, gamma=1.4", "order": "blocked (64 nodes)",
            "ms_per_step": round(ms, 3), "MLUPS": round(N / ms / 1e3, 1), "GBps": round(gbs, 1),
            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "finite": ok and ok_plain,
            "plain_order_ms_per_step": round(ms_plain, 3),
            "pattern_probe_GBps_by_policy": probe, "frac_of_pattern_probe": round(gbs / max(probe.values()), 4)}


def pattern_probe_3d(n, launches=10):
    """The blocked 3-D step's memory pattern with no arithmetic
    (lbm_pattern_probe_3d) on an n^3 grid, ping-pong; GB/s at 2800 B per node
    and launch for each cache policy (default, non-temporal loads,
    non-temporal loads and stores)."""
    import ctypes

    import torch

    from paper_1606_06107_amd import _lib
    lib = _lib.load()
    N = n ** 3
    f = [torch.zeros(343 * N, device="cuda") for _ in range(2)]
    g = [torch.zeros(7 * N, device="cuda") for _ in range(2)]
    stream = torch.cuda.current_stream()
    out = {}

    def launch(k, pol):
        _lib.check(lib.lbm_pattern_probe_3d(pol, ctypes.c_void_p(f[(k + 1) & 1].data_ptr()),
                                            ctypes.c_void_p(f[k & 1].data_ptr()),
                                            ctypes.c_void_p(g[(k + 1) & 1].data_ptr()),
                                            ctypes.c_void_p(g[k & 1].data_ptr()), n, n, n,
                                            ctypes.c_void_p(stream.cuda_stream)))
    for pol, name in ((0, "default"), (1, "nt_loads"), (2, "nt_loads_stores")):
        for k in range(2):
            launch(k, pol)
        a, b = _events(stream)
        torch.cuda.synchronize()
        a.record(stream)
        for k in range(launches):
            launch(k, pol)
        b.record(stream)
        torch.cuda.synchronize()
        out[name] = round(N * 2800 / (a.elapsed_time(b) / launches * 1e-3) / 1e9, 1)
    del f, g
    torch.cuda.empty_cache()
    return out


def extra_3d_full(steps=2000, every=100, tau=None, fp64_gamma=1.4, n=256):
    """The full 3-D workload: 256^3 decaying turbulence, FP32, 2000 steps for
    each gamma of the set (n = 11/3, 2, 0), the kinetic energy every 100
    steps; and the same run in FP64 for one gamma, whose kinetic-energy
    curve the FP32 one is compared with (chaotic flow: no pointwise claim).
    Only the step calls are timed.  Opt-in (--extras turbulence_3d_full):
    about two minutes."""
    import numpy as np
    import torch

    import workloads
    from paper_1606_06107_amd import Sim
    N = n ** 3
    tau = workloads.Turbulence3D().tau if tau is None else tau
    out = {"workload": f"3-D {n}^3 decaying turbulence, D3Q343+D1Q7, tau={tau}, {steps} steps, "
                       "rms Mach 0.3, k^4 exp(-2(k/4)^2) spectrum", "runs": []}
    curves = {}
    for gamma, dt in ((1.3, torch.float32), (1.4, torch.float32), (5.0 / 3.0, torch.float32),
                      (fp64_gamma, torch.float64)):
        w = workloads.Turbulence3D(n=n, gamma=gamma, tau=tau)
        sim = Sim((n,) * 3, n_rot=w.n_rot, tau=tau, dtype=dt).init(*w.fields())
        sim.prepare(every)
        ke, ms, t = [], 0.0, 0
        while True:
            rho, u, T, tot = sim.moments()
            ke.append(float((0.5 * rho * (u * u).sum(0)).sum().item()))
            del rho, u, T
            if t >= steps or not np.isfinite(ke[-1]):
                break
            a, b = _events(sim.stream)
            torch.cuda.synchronize()
            a.record(sim.stream)
            sim.step(every)
            b.record(sim.stream)
            torch.cuda.synchronize()
            ms += a.elapsed_time(b)
            t += every
        name = "f32" if dt == torch.float32 else "f64"
        curves[(round(gamma, 4), name)] = np.array(ke)
        tot = tot.cpu().numpy()
        out["runs"].append({"gamma": round(gamma, 4), "n_rot": round(w.n_rot, 4), "dtype": name,
                            "steps_finite": t if np.isfinite(ke[-1]) else t - every,
                            "ms_per_step": round(ms / max(t, 1), 3), "MLUPS": round(N * t / ms / 1e3, 1),
                            "KE_over_KE0_every_100": [round(v / ke[0], 5) for v in ke],
                            "final_totals": [float(v) for v in tot]})
        print(f"bench: turbulence_3d_full gamma={gamma:.4f} {name} done", file=sys.stderr, flush=True)
        del sim
        torch.cuda.empty_cache()
    a, b = curves.get((round(fp64_gamma, 4), "f32")), curves.get((round(fp64_gamma, 4), "f64"))
    if a is not None and b is not None and len(a) == len(b):
        out["fp32_vs_fp64_KE_max_rel"] = float(np.max(np.abs(a - b) / np.abs(b)))
    return out


def extra_d2q37(steps=200):
    """The paper's own 2-D lattice (D2Q37 of Table I) on the 1024^2 periodic
    workload, FP32, in place, autotuned tile; and the Sec. VI tube
    (1000 x 16, FP64, 180 steps) as a timing of the paper's experiment."""
    import torch

    import workloads
    from paper_1606_06107_amd import Sim
    from paper_1606_06107_amd.autotune import tune_sim
    w = workloads.Periodic2D()
    sim = Sim((w.nx, w.ny), n_rot=w.n_rot, tau=w.tau, dtype=torch.float32, lattice="D2Q37").init(*w.fields())
    tile, _ = tune_sim(sim, steps=20)
    sim.init(*w.fields())
    sim.step(steps)  # warm
    sim.prepare(steps)
    a, b = _events(sim.stream)
    torch.cuda.synchronize()
    a.record(sim.stream)
    sim.step(steps)
    b.record(sim.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    N = w.nx * w.ny
    gbs = N * 2 * (37 + 7) * 4 / (ms * 1e-3) / 1e9
    T = sim.moments(totals=False)[2]
    ok = bool(torch.isfinite(T).all().item())
    del sim, T
    # Sec. VI tube: 1000 x 16, open in x, periodic in y, rho 4:1 at T = 1
    import numpy as np
    Nx, ny, st = 1000, 16, 180
    x = (np.arange(Nx) + 0.5) / Nx
    rho = np.tile(np.where(x < 0.5, 4.0, 1.0), ny)
    tube = Sim((Nx, ny), bc=["open", "periodic"], n_rot=3.0, tau=2.0 / 3.0, dtype=torch.float64,
               lattice="D2Q37")
    tube.init(rho, np.zeros((2, Nx * ny)), np.ones(Nx * ny)).step(st)  # warm
    tube.init(rho, np.zeros((2, Nx * ny)), np.ones(Nx * ny)).prepare(st)
    a, b = _events(tube.stream)
    torch.cuda.synchronize()
    a.record(tube.stream)
    tube.step(st)
    b.record(tube.stream)
    torch.cuda.synchronize()
    ms_tube = a.elapsed_time(b)
    return {"workload": "2-D periodic 1024x1024, D2Q37 (Table I) + D1Q7 FP32, in place, same fields as the headline",
            "tile": list(tile[:2]), "ms_per_step": round(ms, 4), "MLUPS": round(N / ms / 1e3, 1),
            "GBps": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "finite": ok,
            "sec6_tube_1000x16_fp64_180_steps_ms": round(ms_tube, 3)}


def extra_fd(steps=200, courant=0.05):
    """The finite-difference update of Sec. V A (lbm_set_fd) on the 1024^2
    periodic workload, D2Q49 + D1Q7 FP32, Courant factor 0.05 (the largest
    that keeps these fields bounded at tau = 1; the speed does not depend on
    it): each step
    reads every population at its node plus three upwind neighbours per
    axis it moves along (cached) and writes it once."""
    import torch

    import workloads
    from paper_1606_06107_amd import Sim
    w = workloads.Periodic2D()
    sim = Sim((w.nx, w.ny), n_rot=w.n_rot, tau=w.tau, dtype=torch.float32).init(*w.fields()).set_fd(courant)
    sim.step(steps)  # warm
    sim.init(*w.fields()).prepare(steps)
    a, b = _events(sim.stream)
    torch.cuda.synchronize()
    a.record(sim.stream)
    sim.step(steps)
    b.record(sim.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    N = w.nx * w.ny
    gbs = N * 448 / (ms * 1e-3) / 1e9
    T = sim.moments(totals=False)[2]
    ok = bool(torch.isfinite(T).all().item())
    return {"workload": "2-D periodic 1024x1024, D2Q49+D1Q7 FP32, finite-difference update, Courant factor 0.05",
            "ms_per_step": round(ms, 4), "MLUPS": round(N / ms / 1e3, 1), "GBps_algorithmic": round(gbs, 1),
            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "finite": ok}


def extra_transport(tau=0.8, n_values=(0.0, 2.0, 4.0, 6.0)):
    """Shear viscosity and heat diffusivity measured on the GPU (decaying
    Fourier modes, D2Q49 FP64, 64 x 3 periodic) against the Chapman-Enskog
    results: nu = (T/r^2)(tau - 1/2); the paper's kappa implies chi = nu
    (Pr = 1), while only the translational populations carry heat in the
    scheme (chi = (D+2)/(D+n+2) nu)."""
    import torch

    from paper_1606_06107_amd import lattice_info, transport
    r = lattice_info(1)[1]
    nu_th = (tau - 0.5) / r ** 2
    rows = []
    for n in n_values:
        nu = transport.shear_viscosity(n, tau, dtype=torch.float64)
        chi = transport.thermal_diffusivity(n, tau, dtype=torch.float64)
        rows.append({"n": n, "nu": round(nu, 6), "nu_over_theory": round(nu / nu_th, 5), "chi": round(chi, 6),
                     "Pr_measured": round(nu / chi, 4), "Pr_translational_heat_flux": round((n + 4) / 4, 4),
                     "Pr_paper_CE": 1.0})
    return {"workload": "shear and isobaric temperature waves, 64x3 periodic, D2Q49+D1Q7 FP64, tau=0.8, T=1",
            "nu_theory": round(nu_th, 6), "rows": rows}


def extra_batch(seed=0):
    """4096 ragged shock tubes, one persistent launch, FP32 and FP64, with the
    per-instance FP32-vs-FP64 relative L1 error of rho, u, T (Sec. VI)."""
    import numpy as np
    import torch

    import workloads
    from paper_1606_06107_amd import Batch
    from paper_1606_06107_amd.autotune import tune_batch
    bt = workloads.batched_tubes(4096, seed=seed)
    (blk, sup), table = tune_batch(
        lambda b_, s_: Batch(bt.lengths, bt.n_rot, bt.tau, bt.steps, block=b_, superstep=s_),
        (bt.rho, bt.u[0], bt.T), key_extra="tubes4096-f32")
    (blk64, sup64), _ = tune_batch(
        lambda b_, s_: Batch(bt.lengths, bt.n_rot, bt.tau, bt.steps, dtype=torch.float64, block=b_, superstep=s_),
        (bt.rho, bt.u[0], bt.T), supersteps=(16, 24), key_extra="tubes4096-f64")
    out = {"workload": "4096 tubes, L logU[256,8192] (sum 9.26M nodes), D1Q7+D1Q7, one persistent launch",
           "autotuned_block_superstep": [blk, sup], "autotuned_block_superstep_f64": [blk64, sup64]}
    fields = {}
    for name, dt in (("f32", torch.float32), ("f64", torch.float64)):
        kw = dict(block=blk, superstep=sup) if dt == torch.float32 else dict(block=blk64, superstep=sup64)
        b = Batch(bt.lengths, bt.n_rot, bt.tau, bt.steps, dtype=dt, **kw).init(bt.rho, bt.u[0], bt.T)
        b.step()  # graph capture outside the timed region
        b.init(bt.rho, bt.u[0], bt.T)
        a, e = _events(b.stream)
        torch.cuda.synchronize()
        a.record(b.stream)
        b.step()
        e.record(b.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(e)
        st = b.status.cpu().numpy()
        done = b.steps_done.cpu().numpy()
        work = float((bt.lengths * done).sum())
        out[name] = {"ms": round(ms, 2), "node_steps": work, "MLUPS": round(work / ms / 1e3, 1),
                     "status_counts": {str(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}}
        r, u, T = b.moments()
        fields[name] = (st, [b.split(x) for x in (r, u, T)])
        del b
    st32, f32 = fields["f32"]
    st64, f64 = fields["f64"]
    both = np.nonzero((st32 == 0) & (st64 == 0))[0]
    errs = []
    for i in both:
        errs.append([float(np.abs(f32[k][i] - f64[k][i]).sum() / max(np.abs(f64[k][i]).sum(), 1e-300))
                     for k in range(3)])
    errs = np.array(errs) if errs else np.zeros((0, 3))
    out["fp32_vs_fp64_rel_l1"] = {
        "instances": int(len(both)),
        **{f"p{q}_rho_u_T": [float(v) for v in np.percentile(errs, q, axis=0)] for q in (50, 90, 99)},
        "max_rho_u_T": [float(v) for v in errs.max(0)] if len(both) else None,
        "per_instance": "profiles/batched_tubes_4096.md (tests/report_batched_tubes.py)"}
    # the kernel over the FP32-stable tubes alone: every tube runs all its steps
    sub = bt.subset(np.nonzero(st32 == 0)[0])
    b = Batch(sub.lengths, sub.n_rot, sub.tau, sub.steps, block=blk, superstep=sup)
    b.init(sub.rho, sub.u[0], sub.T).step()
    b.init(sub.rho, sub.u[0], sub.T)
    a, e = _events(b.stream)
    torch.cuda.synchronize()
    a.record(b.stream)
    b.step()
    e.record(b.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(e)
    work = float((sub.lengths * sub.steps).sum())
    out["f32_stable_tubes_only"] = {"tubes": int(sub.num), "nodes": int(sub.lengths.sum()), "ms": round(ms, 3),
                                    "node_steps": work, "MLUPS": round(work / ms / 1e3, 1),
                                    "all_completed": bool((b.status.cpu().numpy() == 0).all())}
    return out


def extra_surrogate(train_candidates=262144, test_candidates=4096, test_tubes=256, train_steps=120000, calls=16,
                    pairs_per_tube=16, train_batch=32, lr=2e-3, plain_calls=1, val_tubes=64, val_every=7500):
    """Learned surrogate vs plain LBM on held-out 4096-node tubes: 16 calls
    of k = 16 steps (256 steps) from the initial state; the first
    `plain_calls` calls run the plain scheme (the initial diaphragm is a
    discontinuity), every later one the surrogate with the admission check
    and plain-LBM fallback; errors judged against the plain LBM run (Sec. VI
    relative L1 per tube, averaged over the tubes).  Training data: 262,144
    seeded candidate tubes run by the batch kernel, of which the ~22,000
    that stay stable give 16 pairs each from their initial state (the
    times such a rollout visits); the checkpoint kept is the one with the lowest velocity error of
    the same rollout (no fallback) on `val_tubes` validation tubes drawn
    from a third seed; the admission check's Mach bound is the 99.99th
    percentile over the training pairs of each pair's largest |u|/sqrt(T)
    (predictions outside the trained states go to the plain scheme)."""
    import numpy as np
    import torch

    from paper_1606_06107_amd import Batch, Surrogate
    from paper_1606_06107_amd import surrogate as SG

    def l1(p, q):
        return (torch.abs(p - q).sum(-1) / torch.abs(q).sum(-1).clamp_min(1e-300)).mean(1).cpu().numpy()

    def held_out(seed, n):
        te = SG.stable_tubes(test_candidates, seed=seed)
        te = te.subset(np.arange(min(n, te.num)))
        x0 = torch.as_tensor(np.stack([te.rho, te.u[0], te.T]).reshape(3, te.num, 4096), device="cuda")
        gamma = torch.as_tensor(te.gamma, device="cuda")
        plain = Batch(te.lengths, te.n_rot, te.tau, np.full(te.num, 16 * calls), dtype=torch.float32)
        plain.init(te.rho, te.u[0], te.T)
        # the fallback runs the few rejected tubes' remaining steps, latency-bound:
        # one node per thread in 1024-node chunks, or the rollout's shape for few tubes
        fb = Batch(te.lengths, te.n_rot, te.tau, np.zeros(te.num, dtype=np.int64), dtype=torch.float32,
                   chunk=1024)
        return te, x0, gamma, plain, fb

    t0 = time.perf_counter()
    x, tg, gm, n_stable = SG.training_pairs(train_candidates, seed=0, pairs_per_tube=pairs_per_tube)
    envelope = SG.mach_envelope(x, tg, 0.9999)
    envelope_max = SG.mach_envelope(x, tg, 1.0)
    tv, x0v, gv, plain_v, fbv = held_out(2 * 10 ** 6, val_tubes)
    ref_v = SG.fields_of(plain_v.step()).clone()
    del plain_v
    sur = Surrogate(train_batch, 4096)
    sur.set_params(SG.init_params(0))
    sur_v = sur.shape_like(tv.num)

    def validate():
        xr, _ = SG.rollout(sur_v, x0v, gv, fbv, calls, fallback=False, plain_calls=plain_calls)
        return float(l1(xr, ref_v)[1])
    hist = SG.train(sur, x, tg, gm, steps=train_steps, lr=lr, validate=validate, validate_every=val_every)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del x, tg, sur_v, fbv
    te, x0, gamma, plain, fb = held_out(10 ** 6, test_tubes)
    B = te.num
    plain.step()  # warm (graph capture)
    plain.init(te.rho, te.u[0], te.T)
    a, e = _events(plain.stream)
    torch.cuda.synchronize()
    a.record(plain.stream)
    plain.step()
    e.record(plain.stream)
    torch.cuda.synchronize()
    t_lbm = a.elapsed_time(e)
    ref = SG.fields_of(plain)
    surB = sur.shape_like(B)
    SG.rollout(surB, x0, gamma, fb, calls, plain_calls=plain_calls, max_mach=envelope)  # warm
    a, e = _events(plain.stream)
    torch.cuda.synchronize()
    a.record(plain.stream)
    xr, acc = SG.rollout(surB, x0, gamma, fb, calls, plain_calls=plain_calls, max_mach=envelope)
    e.record(plain.stream)
    torch.cuda.synchronize()
    t_sur = a.elapsed_time(e)
    err, err_id = l1(xr, ref), l1(x0, ref)
    per_tube_u = (torch.abs(xr[1] - ref[1]).sum(-1) / torch.abs(ref[1]).sum(-1)).cpu().numpy()
    xn, _ = SG.rollout(surB, x0, gamma, fb, calls, fallback=False, plain_calls=plain_calls)
    err_nf = l1(xn, ref)
    # tighter Mach bounds: more tubes handed to the plain scheme (restarted from
    # the plain first call, so exact), lower error, more time
    sweep = []
    for bound in (0.6, 0.9, 1.2):
        SG.rollout(surB, x0, gamma, fb, calls, plain_calls=plain_calls, max_mach=bound)  # warm
        a, e = _events(plain.stream)
        torch.cuda.synchronize()
        a.record(plain.stream)
        xm, accm = SG.rollout(surB, x0, gamma, fb, calls, plain_calls=plain_calls, max_mach=bound)
        e.record(plain.stream)
        torch.cuda.synchronize()
        tm = a.elapsed_time(e)
        sweep.append({"max_mach": bound, "rel_l1_rho_u_T": [round(float(v), 5) for v in l1(xm, ref)],
                      "tubes_handed_to_plain_scheme": int(B - int(accm[-1].item())), "ms": round(tm, 3),
                      "speedup": round(t_lbm / tm, 3)})
    xs, _ = SG.rollout(surB, x0, gamma, fb, calls, fallback=False)
    err_all = l1(xs, ref)
    # one call (16 steps) from the initial fields against 16 plain steps
    one = Batch(te.lengths, te.n_rot, te.tau, np.full(B, 16), dtype=torch.float32)
    one.init(te.rho, te.u[0], te.T).step()
    err_one = l1(surB.forward(x0, gamma), SG.fields_of(one))
    err_one_id = l1(x0, SG.fields_of(one))
    # the fused forward alone: 134.7 kFLOP of matrix products per output token
    y = torch.empty_like(x0)
    reps = 20
    a, e = _events(surB.stream)
    torch.cuda.synchronize()
    a.record(surB.stream)
    for _ in range(reps):
        surB.forward(x0, gamma, y)
    e.record(surB.stream)
    torch.cuda.synchronize()
    t_fwd = a.elapsed_time(e) / reps
    fwd_flop = 2.0 * (16 * 64 + 4 * 2 * 64 * 128 + 64 * 12) * B * 1024
    acc_l = [int(v) for v in acc.cpu().tolist()]
    sur_calls = calls - plain_calls
    return {"workload": f"{B} held-out stable 4096-node tubes, {calls} calls x 16 steps, the first "
                        f"{plain_calls} by the plain scheme",
            "train": {"candidate_tubes": train_candidates, "stable_tubes": int(n_stable),
                      "pairs": int(n_stable * pairs_per_tube), "batch": train_batch, "adam_steps": train_steps,
                      "lr": lr, "seconds": round(t_train, 2),
                      "step_loss_validation_u_l1": [[h[0], float(f"{h[1]:.3g}"), round(h[2], 5)] for h in hist],
                      "validation_tubes": int(tv.num)},
            "max_mach_envelope": round(envelope, 4), "training_pairs_max_mach": round(envelope_max, 3),
            "t_lbm_ms": round(t_lbm, 3), "t_surrogate_with_fallback_ms": round(t_sur, 3),
            "speedup": round(t_lbm / t_sur, 3), "plain_calls": plain_calls,
            "surrogate_tube_calls_fraction": round(sum(acc_l) / max(B * sur_calls, 1), 4),
            "tubes_advanced_by_surrogate_per_call": acc_l,
            "tubes_handed_to_plain_scheme": int(B - acc_l[-1]) if acc_l else 0,
            "forward_ms": round(t_fwd, 4),
            "forward_mfma": {"achieved": round(fwd_flop / t_fwd / 1e9, 1), "peak": 2500.0, "unit": "TFLOP/s",
                             "frac": round(fwd_flop / t_fwd / 1e9 / 2500.0, 4)},
            "rel_l1_rho_u_T": [round(float(v), 5) for v in err],
            "u_rel_l1_per_tube": {"median": round(float(np.median(per_tube_u)), 5),
                                  "p90": round(float(np.percentile(per_tube_u, 90)), 5),
                                  "max": round(float(per_tube_u.max()), 5)},
            "rel_l1_no_fallback": [round(float(v), 5) for v in err_nf],
            "mach_bound_sweep": sweep,
            "rel_l1_surrogate_every_call": [round(float(v), 5) for v in err_all],
            "rel_l1_identity": [round(float(v), 5) for v in err_id],
            "one_call_rel_l1": [round(float(v), 5) for v in err_one],
            "one_call_rel_l1_identity": [round(float(v), 5) for v in err_one_id]}


def extra_hbm(steps=40, warmup=10, sizes=((1024, 1024), (4096, 2048))):
    """The headline step at two sizes, in place and ping-pong: 1024^2 (in
    place its 264 MB working set about fits the 256 MB memory-side cache) and
    4096 x 2048 (2.1 GB in place, 3.8 GB ping-pong: 8x / 15x that cache, so
    the memory traffic is HBM traffic).  Autotuned tile per case."""
    import torch

    import workloads
    from paper_1606_06107_amd import Sim
    from paper_1606_06107_amd.autotune import tune_sim
    rows = []
    for nx, ny in sizes:
        w = workloads.Periodic2D(nx=nx, ny=ny)
        fields = w.fields()
        for inplace in (True, False):
            sim = Sim((nx, ny), n_rot=w.n_rot, tau=w.tau, dtype=torch.float32).init(*fields)
            sim.set_inplace(inplace)
            tile, _ = tune_sim(sim, steps=10, reps=3, finalists=2)
            sim.init(*fields)
            sim.step(warmup)
            sim.prepare(steps)
            a, b = _events(sim.stream)
            torch.cuda.synchronize()
            a.record(sim.stream)
            sim.step(steps)
            b.record(sim.stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / steps
            N = nx * ny
            gbs = N * 448 / (ms * 1e-3) / 1e9
            ok = bool(torch.isfinite(sim.moments(totals=False)[2]).all().item())
            ws = N * (49 * (1 if inplace else 2) + 14) * 4
            del sim
            torch.cuda.empty_cache()
            probe = pattern_probe(nx, ny, inplace, steps)
            probe_blk = pattern_probe(nx, ny, inplace, steps, blocked=True)
            best = max(probe.values())
            rows.append({"nodes": f"{nx}x{ny}", "streaming": "in-place" if inplace else "ping-pong",
                         "working_set_MB": round(ws / 1e6, 1), "tile": list(tile[:2]),
                         "ms_per_step": round(ms, 4), "MLUPS": round(N / ms / 1e3, 1), "GBps": round(gbs, 1),
                         "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "finite": ok,
                         "pattern_probe_GBps_by_policy": probe, "frac_of_pattern_probe": round(gbs / best, 4),
                         "pattern_probe_64_node_blocks_GBps_by_policy": probe_blk})
    return {"workload": "headline 2-D step (D2Q49+D1Q7 FP32, 448 B per node-step) at a cache-sized and "
                        "an HBM-sized grid; each beside the memory-only probe of its access pattern "
                        "(lbm_pattern_probe, best of its cache policies), and the probe of the same "
                        "pattern with f in 64-node blocks (not the kernel's layout in 2-D)", "rows": rows}


def extra_placement(holds=8, hold_mb=192, steps=40):
    """The in-place 1024^2 step and its memory-only probe, re-allocated after
    each of `holds` further allocations of `hold_mb` MB (kept alive), so that
    each run lands on other physical pages.  Its 264 MB working set is about
    the size of the 256 MB memory-side cache; whether it stays resident
    depends on where the pages land."""
    import torch

    import workloads
    from paper_1606_06107_amd import Sim
    w = workloads.Periodic2D()
    fields = w.fields()
    N = w.nx * w.ny
    hold, rows = [], []
    for k in range(holds):
        sim = Sim((w.nx, w.ny), n_rot=w.n_rot, tau=w.tau, dtype=torch.float32).init(*fields)
        sim.set_tile(128, 2)
        sim.step(10)
        sim.prepare(steps)
        a, b = _events(sim.stream)
        torch.cuda.synchronize()
        a.record(sim.stream)
        sim.step(steps)
        b.record(sim.stream)
        torch.cuda.synchronize()
        us = a.elapsed_time(b) / steps * 1e3
        del sim
        torch.cuda.empty_cache()
        probe = pattern_probe(w.nx, w.ny, True, steps)
        rows.append({"held_MB": k * hold_mb, "step_us": round(us, 1), "step_GBps": round(N * 448 / us / 1e3, 1),
                     "probe_GBps_by_policy": probe})
        hold.append(torch.empty(hold_mb * 2 ** 20, dtype=torch.uint8, device="cuda"))
    del hold
    torch.cuda.empty_cache()
    return {"workload": "1024^2 in place (D2Q49+D1Q7 FP32, tile 128x2) re-allocated after growing allocations",
            "rows": rows}


def extra_fallback_shapes(demoted=(1, 7, 34, 129), steps=240, reps=6):
    """The surrogate's fallback launch: `steps` plain steps for the first k
    of 256 stable 4096-node tubes (the others have 0 steps), FP32, in the
    fallback batch's own shape (1024-node chunks) and in each shape of
    surrogate.LATENCY_SHAPES; per k the median time of `reps` calls and the
    shape surrogate.latency_shape picks."""
    import numpy as np
    import torch

    from paper_1606_06107_amd import Batch
    from paper_1606_06107_amd import surrogate as SG
    te = SG.stable_tubes(8192, seed=7)
    te = te.subset(np.arange(min(256, te.num)))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    rows = []
    for k in demoted:
        ns = np.zeros(te.num, dtype=np.int64)
        ns[:k] = steps
        b = Batch(te.lengths, te.n_rot, te.tau, ns, dtype=torch.float32, chunk=1024)
        ms = {}
        for c, S in [(0, 0)] + list(SG.LATENCY_SHAPES):
            ts = []
            for r in range(reps + 2):
                b.init(te.rho, te.u[0], te.T)
                a, e = _events(b.stream)
                a.record(b.stream)
                b.step(chunk=c, superstep=S) if c else b.step()
                e.record(b.stream)
                e.synchronize()
                if r >= 2:
                    ts.append(a.elapsed_time(e))
            if not (b.status.cpu().numpy()[:k] == 0).all():
                raise RuntimeError("a fallback tube failed")
            ms[f"{c}x{S}" if c else "1024x24"] = round(float(np.median(ts)), 3)
        b.release()
        pick = SG.latency_shape(k, 4096, cus)
        rows.append({"demoted_tubes": k, "ms_by_chunk_x_superstep": ms,
                     "picked": f"{pick[0]}x{pick[1]}" if pick[0] else "1024x24"})
    return {"workload": f"{steps} steps of k of {te.num} stable 4096-node tubes (the rest 0 steps), FP32 batch kernel",
            "rows": rows}


def pattern_probe(nx, ny, inplace, launches=40, blocked=False):
    """The step's memory pattern with no arithmetic (lbm_pattern_probe) on an
    nx x ny grid: ping-pong (alternating buffers) or in place (even and odd
    launches alternating); GB/s at 448 B per node and launch, for each cache
    policy (default, non-temporal loads of f, non-temporal loads and stores
    of f, non-temporal loads and stores of g only)."""
    import ctypes

    import torch

    from paper_1606_06107_amd import _lib
    lib = _lib.load()
    N = nx * ny
    f = [torch.zeros(49 * N, device="cuda") for _ in range(1 if inplace else 2)]
    g = [torch.zeros(7 * N, device="cuda") for _ in range(2)]
    stream = torch.cuda.current_stream()
    out = {}

    def launch(k, pol):
        if inplace:
            mode, fd, fs = 1 + (k & 1), f[0], f[0]
        else:
            mode, fd, fs = 0, f[(k + 1) & 1], f[k & 1]
        mode += 3 if blocked else 0
        _lib.check(lib.lbm_pattern_probe(mode, pol, ctypes.c_void_p(fd.data_ptr()), ctypes.c_void_p(fs.data_ptr()),
                                         ctypes.c_void_p(g[(k + 1) & 1].data_ptr()),
                                         ctypes.c_void_p(g[k & 1].data_ptr()), nx, ny,
                                         ctypes.c_void_p(stream.cuda_stream)))
    for pol, name in ((0, "default"), (1, "nt_loads"), (2, "nt_loads_stores"), (3, "nt_rotational")):
        for k in range(4):
            launch(k, pol)
        a, b = _events(stream)
        torch.cuda.synchronize()
        a.record(stream)
        for k in range(launches):
            launch(k, pol)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / launches
        out[name] = round(N * 448 / (ms * 1e-3) / 1e9, 1)
    del f, g
    torch.cuda.empty_cache()
    return out


def tile_sweep(nx, ny, steps, inplace):
    """Every compiled 2-D tile for `steps` steps (a profiling aid: under
    rocprofv3 each tile's kernel gets its own statistics line)."""
    import torch

    import workloads
    from paper_1606_06107_amd import Sim
    from paper_1606_06107_amd.autotune import TILES
    w = workloads.Periodic2D(nx=nx, ny=ny)
    sim = Sim((nx, ny), n_rot=w.n_rot, tau=w.tau, dtype=torch.float32).init(*w.fields())
    sim.set_inplace(inplace)
    out = {}
    for t in TILES[2]:
        sim.set_tile(*t)
        sim.prepare(steps)
        a, b = _events(sim.stream)
        torch.cuda.synchronize()
        a.record(sim.stream)
        sim.step(steps)
        b.record(sim.stream)
        torch.cuda.synchronize()
        out["x".join(map(str, t))] = round(1000 * a.elapsed_time(b) / steps, 2)
    print(json.dumps({"tile_sweep_us_per_step": out, "nodes": f"{nx}x{ny}",
                      "streaming": "in-place" if inplace else "ping-pong"}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=1024)
    ap.add_argument("--monitor-every", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--tile", type=str, default="")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", type=str,
                    default="hbm,tube_1d,turbulence_3d,d2q37,fd,transport,batched_tubes,surrogate",
                    help="comma-separated subset of the extra workloads to run (opt-in, not in the "
                         "default: turbulence_3d_full, placement, fallback_shapes)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--sur-train-steps", type=int, default=120000,
                    help="Adam steps of the surrogate extra's training")
    ap.add_argument("--sur-train-candidates", type=int, default=262144,
                    help="seeded tubes generated for the surrogate's training (the stable ones are used)")
    ap.add_argument("--ping-pong", action="store_true",
                    help="two translational buffers instead of in-place streaming")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="first run a plain device copy of this many MB (5 times): the reference "
                         "kernel for scaling HBM traffic counters")
    ap.add_argument("--tile-sweep", action="store_true",
                    help="only run every compiled 2-D tile for --steps steps (for profiling) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the benchmark runs on one GPU "
              "(the multi-GPU sharding of the step is not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_1606_06107_amd import Sim

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * 1024 * 1024 // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.tile_sweep:
        tile_sweep(args.nx, args.ny, args.steps, not args.ping_pong)
        return
    w = workloads.Periodic2D(nx=args.nx, ny=args.ny)
    rho, u, T = w.fields()
    N = args.nx * args.ny
    sim = Sim((args.nx, args.ny), n_rot=w.n_rot, tau=w.tau, dtype=torch.float32).init(rho, u, T)
    sim_inplace = not args.ping_pong
    sim.set_inplace(sim_inplace)
    tuned, tune_table = None, None
    if args.tile:
        sim.set_tile(*[int(v) for v in args.tile.split("x")])
    elif not args.no_autotune:
        from paper_1606_06107_amd.autotune import tune_sim
        tuned, tune_table = tune_sim(sim, steps=20)
        sim.init(rho, u, T)  # tuning advanced the state; start over
    total_steps = args.warmup + args.steps
    cap = total_steps // args.monitor_every + 2
    series = sim.set_monitor(args.monitor_every, cap)
    sim.step(args.warmup)
    sim.prepare(args.steps)  # the timed call's graph is recorded before timing
    stream = sim.stream
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    t0 = time.perf_counter()
    sim.step(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    ms_per_step = ms / args.steps

    # correctness of the run: finite fields and FP64 conservation totals
    _, _, Tn, tot = sim.moments()
    torch.cuda.synchronize()
    s = series.cpu().numpy()
    s = s[np.isfinite(s[:, 0])]
    tot = tot.cpu().numpy()
    mass_drift = float(abs(tot[0] - s[0, 0]) / s[0, 0])
    mom_drift = float(np.abs(tot[1:3] - s[0, 1:3]).max() / s[0, 0])
    energy_drift = float(abs(tot[3] - s[0, 3]) / s[0, 3])
    finite = bool(torch.isfinite(Tn).all().item())

    used_tile = tuple(tuned) if tuned else (
        tuple(int(v) for v in args.tile.split("x")) if args.tile else (256, 1))
    traffic = TRAFFIC["bytes"].get(tuple(used_tile)) if (
        kernel_sha() == TRAFFIC["sha256"] and N == TRAFFIC["nodes"] and sim_inplace) else None
    mlups = N / (ms_per_step * 1e-3) / 1e6
    bytes_per_node = 2 * (49 + 7) * 4  # read + write every population once
    achieved_gbs = N * bytes_per_node / (ms_per_step * 1e-3) / 1e9
    del sim
    torch.cuda.empty_cache()
    copy = copy_bandwidth(2048)  # 2 GB each way: well beyond the memory-side cache
    copy_gbs = copy["lbm_stream_copy"]
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2-D periodic compressible flow, D2Q49+D1Q7, {args.nx}x{args.ny} "
                               f"nodes, FP32 populations / FP64 moments, gamma=1.4 (n=3), "
                               f"tau=1, 8-mode random fields at Mach 0.3, seed 0, "
                               f"FP64 totals every {args.monitor_every} steps",
                   "streaming": "in-place" if sim_inplace else "ping-pong",
                   "nodes": N, "bytes_per_node_step": bytes_per_node,
                   "tile": list(used_tile)},
        "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "copy_GBps": copy_gbs, "torch_copy_GBps": copy["torch"],
                     "frac_of_copy": round(achieved_gbs / copy_gbs, 4)},
        "checks": {"finite": finite, "mass_drift": mass_drift, "momentum_drift": mom_drift,
                   "energy_drift_n3": energy_drift, "wall_s": round(wall, 3)},
    }
    if tune_table is not None:
        out["autotune"] = tune_table
    if not args.no_extras:
        extra = {}
        wanted = set(args.extras.split(","))
        for name, fn in (("hbm", extra_hbm), ("tube_1d", extra_tube_1d), ("turbulence_3d", extra_3d),
                         ("turbulence_3d_full", extra_3d_full), ("placement", extra_placement),
                         ("fallback_shapes", extra_fallback_shapes),
                         ("d2q37", extra_d2q37), ("fd", extra_fd),
                         ("transport", extra_transport), ("batched_tubes", extra_batch),
                         ("surrogate", lambda: extra_surrogate(train_steps=args.sur_train_steps,
                                                               train_candidates=args.sur_train_candidates))):
            if name not in wanted:
                continue
            print(f"bench: {name}", file=sys.stderr, flush=True)
            extra[name] = fn()
            torch.cuda.empty_cache()
        for row in extra.get("hbm", {}).get("rows", []):
            row["frac_of_copy"] = round(row["GBps"] / copy_gbs, 4)
        out["extra"] = extra
    if not args.no_cpu_baseline:
        threads = min(16, len(os.sched_getaffinity(0)))
        print("bench: cpu_baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.nx, args.ny, args.cpu_steps, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
