"""The largest grids the library accepts (N * sizeof(population) just under
2^32 bytes per population row; N < 2^30 nodes in FP32, < 2^29 in FP64):
a 1-D open tube of that length, 4 steps, against the FP64 oracle on windows
at its start, middle and end.  After k steps a node depends only on nodes
within 3k (streaming) of it, so an oracle run on the window widened by a
margin of more than 3k nodes gives the exact values in the window; the
windows at the tube's ends include its open ends.  Needs ~175 GB of device
memory."""
import numpy as np
import pytest

import oracle
from gpu_helpers import announce

pytestmark = pytest.mark.gpu

STEPS = 4
MARGIN = 3 * STEPS + 8
TOL = {"float32": 1e-5, "float64": 1e-12}


def _fields(x, mod=np.mod, sin=np.sin, cos=np.cos):
    """Smooth initial fields as functions of the global node index (FP64).
    The index is reduced modulo each period first (exact for integers), so
    that sin and cos only see arguments in [0, 2 pi): the host's and the
    device's large-argument reductions need not agree to the last bits."""
    two_pi = 2.0 * np.pi
    rho = 1.0 + 0.1 * sin(two_pi * mod(x, 997.0) / 997.0)
    u = 0.1 * sin(two_pi * mod(x, 1009.0) / 1009.0)
    T = 1.0 + 0.05 * cos(two_pi * mod(x, 1013.0) / 1013.0)
    return rho, u, T


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_largest_1d_tube_matches_oracle_windows(dtype_name):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06107_amd import Sim
    dtype = getattr(torch, dtype_name)
    size = 4 if dtype_name == "float32" else 8
    N = (1 << 32) // size - 1
    N = min(N, (1 << 31) - 1)
    free, _ = torch.cuda.mem_get_info()
    need = 4 * 7 * N * size + 6 * 8 * N
    if free < need * 1.1:
        pytest.skip(f"needs {need / 1e9:.0f} GB of device memory, {free / 1e9:.0f} GB free")
    announce(f"largest 1-D tube {dtype_name} N={N} x {STEPS} steps")
    x = torch.arange(N, dtype=torch.float64, device="cuda")
    rho, u, T = _fields(x, torch.remainder, torch.sin, torch.cos)
    del x
    sim = Sim((N,), bc=["open"], n_rot=2.0, tau=0.8, dtype=dtype).init(rho, u.reshape(1, N), T)
    del rho, u, T
    sim.step(STEPS)
    r_d, u_d, T_d, _ = sim.moments(totals=False)
    torch.cuda.synchronize()
    for a, b in ((0, 300), (N // 2 - 150, N // 2 + 150), (N - 300, N)):
        lo, hi = max(0, a - MARGIN), min(N, b + MARGIN)
        xs = np.arange(lo, hi, dtype=np.float64)
        G = oracle.Grid(oracle.D1Q7, (hi - lo,), bc=(oracle.OPEN,), n_rot=2.0, tau=0.8)
        r0, u0, T0 = _fields(xs)
        f, g = G.init_eq(r0, u0.reshape(1, -1), T0)
        G.step(f, g, STEPS)
        orr, oru, orT = G.moments(f, g)[:3]
        # nodes whose 3k-neighbourhood lies inside [lo, hi) or reaches a real end
        keep_lo = a - lo if lo == 0 else max(a - lo, MARGIN)
        keep_hi = (b - lo) if hi == N else min(b - lo, hi - lo - MARGIN)
        sl = slice(keep_lo, keep_hi)
        gr = [t[lo:hi].cpu().numpy()[sl] for t in (r_d, u_d[0], T_d)]
        err = max(float(np.abs(gr[0] - orr[sl]).max()), float(np.abs(gr[1] - oru[0][sl]).max()),
                  float(np.abs(gr[2] - orT[sl]).max()))
        print(f"window [{a}, {b}): L-inf {err:.2e}", flush=True)
        assert err <= TOL[dtype_name], (a, b, err)
    del sim, r_d, u_d, T_d
    torch.cuda.empty_cache()


def _windows(lo_tube, n, a, b):
    """Oracle range [lo, hi) around window [a, b) of an n-node tube and the
    slice of it (relative to lo) that the range's artificial edges cannot
    reach within STEPS steps."""
    lo, hi = max(0, a - MARGIN), min(n, b + MARGIN)
    keep_lo = a - lo if lo == 0 else max(a - lo, MARGIN)
    keep_hi = (b - lo) if hi == n else min(b - lo, hi - lo - MARGIN)
    return lo, hi, slice(keep_lo, keep_hi)


def test_batch_beyond_2_30_nodes_matches_oracle_windows():
    """Three 400 M-node tubes and a 1000-node one (1.2e9 nodes, FP32 rows of
    4.8 GB) in one persistent launch, per-tube n and tau, 4 steps: oracle
    windows at each long tube's start, middle and end, and the short tube
    whole."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06107_amd import Batch
    lengths = np.array([400_000_000, 400_000_000, 400_000_003, 1000], dtype=np.int64)
    n_rot = np.array([2.0, 3.0, 1.5, 4.0])
    tau = np.array([0.8, 0.9, 0.7, 1.0])
    total = int(lengths.sum())
    free, _ = torch.cuda.mem_get_info()
    need = 4 * 7 * total * 4 + 6 * 8 * total
    if free < need * 1.15:
        pytest.skip(f"needs {need / 1e9:.0f} GB of device memory, {free / 1e9:.0f} GB free")
    announce(f"batch of {len(lengths)} tubes, {total} nodes, FP32 x {STEPS} steps")
    x = torch.arange(total, dtype=torch.float64, device="cuda")
    rho, u, T = _fields(x, torch.remainder, torch.sin, torch.cos)
    del x
    b = Batch(lengths, n_rot, tau, np.full(len(lengths), STEPS), dtype=torch.float32).init(rho, u, T)
    del rho, u, T
    b.step()
    st = b.status.cpu().numpy()
    assert (st == 0).all(), st
    r_d, u_d, T_d = b.moments()
    torch.cuda.synchronize()
    off = b.offsets_h
    for i, n in enumerate(lengths):
        n = int(n)
        wins = [(0, n)] if n <= 1000 else [(0, 300), (n // 2 - 150, n // 2 + 150), (n - 300, n)]
        for a, bb in wins:
            lo, hi, sl = _windows(0, n, a, bb)
            xs = np.arange(off[i] + lo, off[i] + hi, dtype=np.float64)
            G = oracle.Grid(oracle.D1Q7, (hi - lo,), bc=(oracle.OPEN,), n_rot=float(n_rot[i]), tau=float(tau[i]))
            r0, u0, T0 = _fields(xs)
            f, g = G.init_eq(r0, u0.reshape(1, -1), T0)
            G.step(f, g, STEPS)
            orr, oru, orT = G.moments(f, g)[:3]
            gr = [t[off[i] + lo:off[i] + hi].cpu().numpy()[sl] for t in (r_d, u_d, T_d)]
            err = max(float(np.abs(gr[0] - orr[sl]).max()), float(np.abs(gr[1] - oru[0][sl]).max()),
                      float(np.abs(gr[2] - orT[sl]).max()))
            print(f"tube {i} window [{a}, {bb}): L-inf {err:.2e}", flush=True)
            assert err <= TOL["float32"], (i, a, bb, err)
    b.release()
    del b, r_d, u_d, T_d
    torch.cuda.empty_cache()
