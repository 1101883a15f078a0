"""Per-instance report of the batched shock-tube workload (4096 tubes, lengths
log-uniform in [256, 8192], per-tube gamma, tau, pressure and density
ratios), run on the GPU by the persistent batch kernel in FP32 and FP64.

For every tube that stays positive in both precisions: the relative L1
error (Sec. VI) of FP32 against FP64 in rho, u, T, and of FP64 against the
exact Riemann solution (oracle/riemann.py) in rho, u, p, T at the tube's end
time.  For every tube that stops (status 2: rho <= 0 or T <= 0, or 1:
non-finite): the cause, read from the exact solution -- the rotational
Courant number |u*| / r of the star state against the linear stability
limit of the forward-Euler upwind update at the tube's omega = 1/tau, and
the sign of the fourth-order translational equilibrium at the two star
states of the exact solution.  Plus the batch kernel's throughput over the stable tubes
alone, and the same tubes with the rotational advection in 2, 4 and 8
sub-steps.

Not collected by pytest (a GPU report, not a test).  Usage, from the
repository root on a GPU machine:

    python tests/report_batched_tubes.py out/batched_tubes_4096.md

The per-instance table of the stable tubes goes to the .csv of the same
name beside the given path (it is too long for the summary)."""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle import riemann  # noqa: E402
from oracle.metrics import l1_rel_error  # noqa: E402


def courant_limit(omega):
    """Largest nu with |1 - omega - nu s(theta)| <= 1 for all theta, s the
    Fourier symbol of the third-order upwind difference (nu >= 0 branch)."""
    th = np.linspace(0.0, np.pi, 20001)
    s = (np.exp(-2j * th) - 6.0 * np.exp(-1j * th) + 3.0 + 2.0 * np.exp(1j * th)) / 6.0
    lo, hi = 0.0, 3.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if np.abs(1.0 - omega - mid * s).max() <= 1.0 + 1e-12:
            lo = mid
        else:
            hi = mid
    return lo


def exact_states(left, right, gamma, n=51):
    """(rho, u, p) samples across the exact solution's wave fan (the star
    region, both rarefactions or shocks, and the initial states)."""
    ps, us, rl, rr = riemann.star_state(left, right, gamma)
    cl = np.sqrt(gamma * left[2] / left[0])
    cr = np.sqrt(gamma * right[2] / right[0])
    s = np.linspace(left[1] - 1.5 * cl, right[1] + 1.5 * cr, n)
    r, u, p = riemann.sample(left, right, gamma, s)
    return r, u, p, (ps, us, rl, rr)


def main(out_md):
    import torch

    from paper_1606_06107_amd import Batch
    r_lat = oracle.d1q7_r()
    bt = workloads.batched_tubes(4096, seed=0)
    I = bt.num
    runs = {}
    for name, dt, blk in (("f32", torch.float32, 1024), ("f64", torch.float64, 512)):
        b = Batch(bt.lengths, bt.n_rot, bt.tau, bt.steps, dtype=dt, block=blk, superstep=24)
        b.init(bt.rho, bt.u[0], bt.T).step()
        torch.cuda.synchronize()
        st = b.status.cpu().numpy()
        done = b.steps_done.cpu().numpy()
        r, u, T = b.moments()
        runs[name] = (st, done, [b.split(x) for x in (r, u, T)])
        b.release()
        del b
        torch.cuda.empty_cache()
        print(f"{name}: status counts {dict(zip(*np.unique(st, return_counts=True)))}", flush=True)
    st32, _, f32 = runs["f32"]
    st64, done64, f64 = runs["f64"]

    # stable tubes: FP32 vs FP64 and FP64 vs the exact solution at t = steps / (L r)
    rows = []
    both = np.nonzero((st32 == 0) & (st64 == 0))[0]
    for i in both:
        L = int(bt.lengths[i])
        e32 = [l1_rel_error(f32[k][i], f64[k][i]) for k in range(3)]
        t = float(bt.steps[i]) / (L * r_lat)
        x = (np.arange(L) + 0.5) / L
        left, right = tuple(bt.left[i]), tuple(bt.right[i])
        ra, ua, pa = riemann.sample(left, right, float(bt.gamma[i]), (x - 0.5) / t)
        rho, u, T = f64[0][i], f64[1][i], f64[2][i]
        ex = [l1_rel_error(rho, ra), l1_rel_error(u, ua), l1_rel_error(rho * T, pa), l1_rel_error(T, pa / ra)]
        rows.append((int(i), L, float(bt.gamma[i]), float(bt.tau[i]), float(left[2] / right[2]),
                     float(left[0] / right[0]), int(bt.steps[i]), *e32, *ex))
    rows = np.array(rows)

    # failed tubes (in FP64): cause from the exact solution
    failed = np.nonzero(st64 != 0)[0]
    limits = {}
    cls = {"rotational Courant limit only": 0, "translational equilibrium negative only": 0, "both": 0,
           "neither": 0}
    nu_over = []
    for i in failed:
        left, right, gm = tuple(bt.left[i]), tuple(bt.right[i]), float(bt.gamma[i])
        om = round(1.0 / float(bt.tau[i]), 3)
        if om not in limits:
            limits[om] = courant_limit(om)
        r, u, p, (ps, us, rl, rr) = exact_states(left, right, gm)
        nu = np.abs(u).max() / r_lat
        nu_over.append(nu / limits[om])
        # the two star plateaus, which persist and grow with time
        neg = any(oracle.feq(oracle.D1Q7, 1.0, [us], ps / rs).min() < 0.0 for rs in (rl, rr))
        courant = nu > limits[om]
        key = ("both" if neg else "rotational Courant limit only") if courant else (
            "translational equilibrium negative only" if neg else "neither")
        cls[key] += 1
    stable_nu = []
    for i in both:
        left, right, gm = tuple(bt.left[i]), tuple(bt.right[i]), float(bt.gamma[i])
        om = round(1.0 / float(bt.tau[i]), 3)
        if om not in limits:
            limits[om] = courant_limit(om)
        _, u, _, _ = exact_states(left, right, gm)
        stable_nu.append(np.abs(u).max() / r_lat / limits[om])

    # the batch kernel over the stable tubes alone (FP32)
    sub = bt.subset(np.nonzero(st32 == 0)[0])
    b = Batch(sub.lengths, sub.n_rot, sub.tau, sub.steps, dtype=torch.float32, block=1024, superstep=24)
    b.init(sub.rho, sub.u[0], sub.T).step()
    b.init(sub.rho, sub.u[0], sub.T)
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(b.stream)
    b.step()
    e.record(b.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(e)
    work = float((sub.lengths * sub.steps).sum())
    assert (b.status.cpu().numpy() == 0).all()

    # the same tubes with the rotational advection in m sub-steps (g_substeps):
    # FP64 status and accuracy against the exact solution, FP32 time over the
    # tubes that complete
    subrows = []
    for m in (2, 4, 8):
        b = Batch(bt.lengths, bt.n_rot, bt.tau, bt.steps, dtype=torch.float64, block=512, g_substeps=m)
        b.init(bt.rho, bt.u[0], bt.T).step()
        torch.cuda.synchronize()
        stm = b.status.cpu().numpy()
        r, u, T = b.moments()
        fm = [b.split(x) for x in (r, u, T)]
        b.release()
        del b
        ok = np.nonzero(stm == 0)[0]
        ex_m = []
        for i in ok:
            L = int(bt.lengths[i])
            t = float(bt.steps[i]) / (L * r_lat)
            x = (np.arange(L) + 0.5) / L
            ra, ua, pa = riemann.sample(tuple(bt.left[i]), tuple(bt.right[i]), float(bt.gamma[i]), (x - 0.5) / t)
            ex_m.append([l1_rel_error(fm[0][i], ra), l1_rel_error(fm[1][i], ua),
                         l1_rel_error(fm[0][i] * fm[2][i], pa)])
        ex_m = np.array(ex_m)
        rescued = int(((stm == 0) & (st64 != 0)).sum())
        lost = int(((stm != 0) & (st64 == 0)).sum())
        sm = bt.subset(ok)
        b = Batch(sm.lengths, sm.n_rot, sm.tau, sm.steps, dtype=torch.float32, block=1024, g_substeps=m)
        b.init(sm.rho, sm.u[0], sm.T).step()
        b.init(sm.rho, sm.u[0], sm.T)
        a_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a_.record(b.stream)
        b.step()
        e_.record(b.stream)
        torch.cuda.synchronize()
        ms_m = a_.elapsed_time(e_)
        n32 = int((b.status.cpu().numpy() == 0).sum())
        work_m = float((sm.lengths * b.steps_done.cpu().numpy()).sum())  # steps actually executed
        b.release()
        del b
        torch.cuda.empty_cache()
        subrows.append((m, len(ok), rescued, lost, np.median(ex_m, 0), np.percentile(ex_m, 90, 0), n32, ms_m,
                        work_m))
        print(f"g_substeps {m}: {len(ok)} FP64-stable ({rescued} rescued, {lost} lost), FP32 {n32} of them, "
              f"{ms_m:.2f} ms", flush=True)

    pct = lambda col: [float(np.percentile(rows[:, col], q)) for q in (50, 90, 99, 100)]
    lines = [
        "# Batched shock tubes (4096 tubes): per-instance errors and failure causes",
        "",
        "Workload: `workloads.batched_tubes(4096, seed=0)` -- lengths log-uniform in [256, 8192] "
        f"(sum {int(bt.lengths.sum()):,} nodes), gamma U[1.1, 1.67], tau U[0.6, 1], pressure ratio "
        "logU[2, 100], density ratio U[1, 10], steps = 0.8 of the fastest wave's exit time.  "
        "Persistent batch kernel, FP32 (block 1024, superstep 24) and FP64 (block 512, superstep 24).",
        "",
        "Command (repo root, MI355X):",
        "",
        "```",
        f"python tests/report_batched_tubes.py {out_md}",
        "```",
        "",
        "## Status",
        "",
        f"| | FP32 | FP64 |",
        f"|---|---|---|",
        f"| 0 (completed) | {(st32 == 0).sum()} | {(st64 == 0).sum()} |",
        f"| 1 (non-finite) | {(st32 == 1).sum()} | {(st64 == 1).sum()} |",
        f"| 2 (rho <= 0 or T <= 0) | {(st32 == 2).sum()} | {(st64 == 2).sum()} |",
        "",
        "## Stable tubes (completed in both precisions): relative L1 (Sec. VI), percentiles over "
        f"{len(rows)} tubes",
        "",
        "| | p50 | p90 | p99 | max |",
        "|---|---|---|---|---|",
    ]
    for name, col in (("FP32 vs FP64, rho", 7), ("FP32 vs FP64, u", 8), ("FP32 vs FP64, T", 9),
                      ("FP64 vs exact Riemann, rho", 10), ("FP64 vs exact Riemann, u", 11),
                      ("FP64 vs exact Riemann, p", 12), ("FP64 vs exact Riemann, T", 13)):
        lines.append(f"| {name} | " + " | ".join(f"{v:.2e}" for v in pct(col)) + " |")
    worst = rows[np.argsort(-rows[:, 8])[:5]]
    lines += ["", "Largest FP32-vs-FP64 velocity errors (tube, L, gamma, tau, pressure ratio, density ratio, "
              "steps: FP32-vs-FP64 rho/u/T; FP64-vs-exact rho/u/p/T):", ""]
    for w_ in worst:
        lines.append(f"- tube {int(w_[0])}, L {int(w_[1])}, gamma {w_[2]:.3f}, tau {w_[3]:.2f}, pr {w_[4]:.1f}, "
                     f"dr {w_[5]:.2f}, {int(w_[6])} steps: {w_[7]:.1e} / {w_[8]:.1e} / {w_[9]:.1e}; "
                     f"{w_[10]:.1e} / {w_[11]:.1e} / {w_[12]:.1e} / {w_[13]:.1e}")
    lines += ["", f"## Failed tubes (FP64, {len(failed)}): cause read from the exact solution", "",
              "Rotational Courant number nu* = max |u| / r over the exact solution against the linear "
              "stability limit of the forward-Euler third-order upwind update at omega = 1/tau "
              "(largest nu with |1 - omega - nu s(theta)| <= 1 for every Fourier mode; 0.667 at omega = 1, "
              "0.375 at 1.5, 0.25 at 1.67); translational equilibrium (fourth-order D1Q7) evaluated at "
              "the two star states of the exact solution.", "",
              "| class | tubes |", "|---|---|"]
    for k, v in cls.items():
        lines.append(f"| {k} | {v} |")
    nu_over = np.array(nu_over)
    stable_nu = np.array(stable_nu)
    lines += ["",
              f"nu* / limit: failed tubes median {np.median(nu_over):.2f} (p10 {np.percentile(nu_over, 10):.2f}); "
              f"stable tubes median {np.median(stable_nu):.2f} (p90 {np.percentile(stable_nu, 90):.2f}, "
              f"max {stable_nu.max():.2f}).",
              "",
              "## Throughput",
              "",
              f"The batch kernel over the {sub.num} FP32-stable tubes alone: {ms:.2f} ms for {work:.3e} node-steps "
              f"= {work / ms / 1e3:,.0f} MLUPS (the all-tube launch stops most tubes early; its MLUPS counts "
              "the steps actually executed).",
              "",
              "## Rotational advection in m sub-steps (`g_substeps`)",
              "",
              "The same 4096 tubes with the rotational populations advected in m sub-steps of c/m per "
              "time step (relaxation once per step), FP64 (block 512): tubes that complete, tubes that "
              "complete now but not as written (rescued) and the reverse (lost), the FP64-vs-exact "
              "relative L1 of rho / u / p over the completed tubes, and the FP32 kernel over those tubes "
              "(block 1024; how many complete in FP32, its time and rate).",
              "",
              "| m | FP64 completed | rescued | lost | exact L1 p50 rho / u / p | exact L1 p90 rho / u / p "
              "| FP32 completed | FP32 ms | MLUPS |",
              "|---|---|---|---|---|---|---|---|---|"]
    for m, n_ok, resc, lost, p50, p90, n32, ms_m, work_m in subrows:
        lines.append(f"| {m} | {n_ok} | {resc} | {lost} | " + " / ".join(f"{v:.2e}" for v in p50) + " | "
                     + " / ".join(f"{v:.2e}" for v in p90) + f" | {n32} | {ms_m:.2f} | {work_m / ms_m / 1e3:,.0f} |")
    os.makedirs(os.path.dirname(os.path.join(ROOT, out_md)), exist_ok=True)
    with open(os.path.join(ROOT, out_md), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    csv = os.path.splitext(os.path.join(ROOT, out_md))[0] + ".csv"
    header = ("tube,L,gamma,tau,pressure_ratio,density_ratio,steps,l1_f32_f64_rho,l1_f32_f64_u,l1_f32_f64_T,"
              "l1_exact_rho,l1_exact_u,l1_exact_p,l1_exact_T")
    np.savetxt(csv, rows, delimiter=",", header=header, comments="",
               fmt=["%d", "%d", "%.4f", "%.3f", "%.3f", "%.3f", "%d"] + ["%.3e"] * 7)
    print("\n".join(lines), flush=True)


if __name__ == "__main__":
    t0 = time.time()
    main(sys.argv[1] if len(sys.argv) > 1 else "profiles/batched_tubes_4096.md")
    print(f"report done in {time.time() - t0:.1f} s", flush=True)
