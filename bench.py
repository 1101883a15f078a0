"""Benchmark of the decoupled Hermite lattice Boltzmann hot path on one GPU.

Workload (the metric's configuration): 2-D periodic compressible flow on
D2Q49 (translational) + D1Q7 (rotational), 1024 x 1024 nodes, FP32
populations with FP64 moments/temperature, gamma = 1.4 (n = 3), tau = 1,
seeded smooth random fields with Mach 0.3, conservation totals reduced in
FP64 every 100 steps (fused into the step).  One "step" = one time step of
the whole grid.  Inputs are resident in HBM before timing.

Prints ONE JSON line (rank 0).  --gpus N > 1 is not supported: this build
runs on a single GPU.
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
METRIC = "MLUPS & % HBM roofline; surrogate vs plain LBM speedup at <=1e-2 L1 error"


def cpu_baseline(nx, ny, steps, threads):
    """The CPU oracle (plain C, FP64) on a bounded sample of the same workload."""
    import numpy as np

    import oracle
    import workloads
    used = oracle.set_threads(threads)
    w = workloads.Periodic2D(nx=nx, ny=ny)
    rho, u, T = w.fields()
    G = oracle.Grid(oracle.D2Q49, (nx, ny), n_rot=w.n_rot, tau=w.tau)
    f, g = G.init_eq(rho, u, T)
    G.step(f, g, 1)  # warm-up (page faults, thread start)
    t0 = time.perf_counter()
    G.step(f, g, steps)
    dt = time.perf_counter() - t0
    assert np.isfinite(f).all()
    return {"value": round(nx * ny * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": used,
            "kind": "oracle",
            "sample": f"{nx}x{ny} nodes x {steps} steps of the same 2-D workload, FP64, "
                      f"{dt:.1f} s wall"}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build measures one GPU "
              "(see DESIGN.md for how the path would shard).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_1606_06107_amd import Sim

    torch.cuda.set_device(0)
    w = workloads.Periodic2D(nx=args.nx, ny=args.ny)
    rho, u, T = w.fields()
    N = args.nx * args.ny
    sim = Sim((args.nx, args.ny), n_rot=w.n_rot, tau=w.tau, dtype=torch.float32).init(rho, u, T)
    if args.tile:
        sim.set_tile(*[int(v) for v in args.tile.split("x")])
    total_steps = args.warmup + args.steps
    cap = total_steps // args.monitor_every + 2
    series = sim.set_monitor(args.monitor_every, cap)
    sim.step(args.warmup)
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

    mlups = N / (ms_per_step * 1e-3) / 1e6
    bytes_per_node = 2 * (49 + 7) * 4  # read + write every population once
    achieved_gbs = N * bytes_per_node / (ms_per_step * 1e-3) / 1e9
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
                   "nodes": N, "bytes_per_node_step": bytes_per_node},
        "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "checks": {"finite": finite, "mass_drift": mass_drift, "momentum_drift": mom_drift,
                   "energy_drift_n3": energy_drift, "wall_s": round(wall, 3)},
    }
    if not args.no_cpu_baseline:
        threads = min(16, len(os.sched_getaffinity(0)))
        out["cpu_baseline"] = cpu_baseline(args.nx, args.ny, args.cpu_steps, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
