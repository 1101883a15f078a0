"""GPU parity of the batched persistent launch (lbm_batch_*) against the CPU
oracle run tube by tube, plus scheduling properties."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


LENGTHS = [5, 17, 64, 100, 255, 300, 513, 700, 1024, 1500, 2000, 2500]


def _mild_batch(seed, lengths=LENGTHS):
    """Stable shock tubes: pressure ratio 1.5-4, density ratio 1-3."""
    rng = np.random.default_rng(seed)
    I = len(lengths)
    gamma = rng.uniform(1.2, 1.6, I)
    n_rot = workloads.n_of_gamma(gamma, 1)
    tau = rng.uniform(0.7, 1.0, I)
    steps = rng.integers(20, 90, I)
    pr = rng.uniform(1.5, 4.0, I)
    dr = rng.uniform(1.0, 3.0, I)
    fields = [workloads.sod_tube(L, (1.0, 0.0, 1.0), (1.0 / d, 0.0, 1.0 / p))
              for L, d, p in zip(lengths, dr, pr)]
    rho = np.concatenate([f[0] for f in fields])
    u = np.concatenate([f[1][0] for f in fields])
    T = np.concatenate([f[2] for f in fields])
    return n_rot, tau, steps, rho, u, T, fields


def _oracle_tube(fields, n_rot, tau, steps, g_substeps=1):
    rho, u, T = fields
    G = oracle.Grid(oracle.D1Q7, (len(rho),), bc=(oracle.OPEN,), n_rot=n_rot, tau=tau, g_substeps=g_substeps)
    f, g = G.init_eq(rho, u, T)
    G.step(f, g, steps)
    return G.moments(f, g)[:3]


@pytest.mark.parametrize("dtype,chunk,superstep,m", [("float64", 0, 0, 1), ("float64", 256, 8, 1),
                                                     ("float32", 0, 0, 1), ("float32", 448, 16, 1),
                                                     ("float64", 0, 0, 4), ("float64", 512, 6, 3),
                                                     ("float32", 0, 0, 4), ("float32", 640, 8, 5)])
def test_batch_matches_oracle_per_tube(torch_cuda, dtype, chunk, superstep, m):
    """chunk=0: the library's capacity (most tubes on chip in one piece);
    small chunks force the halo'd multi-pass path for the long tubes.  m > 1:
    the rotational advection in m sub-steps (halos of max(3, 2m) nodes per
    step), against the oracle's sub-stepped update."""
    from paper_1606_06107_amd import Batch
    announce(f"batch {dtype} chunk={chunk} superstep={superstep} g_substeps={m}")
    n_rot, tau, steps, rho, u, T, fields = _mild_batch(1)
    b = Batch(LENGTHS, n_rot, tau, steps, dtype=getattr(torch_cuda, dtype), chunk=chunk,
              superstep=superstep, g_substeps=m).init(rho, u, T)
    b.step()
    r, uu, TT = b.moments()
    torch_cuda.cuda.synchronize()
    assert (b.status.cpu().numpy() == 0).all()
    R, U, Tt = b.split(r), b.split(uu), b.split(TT)
    for i, L in enumerate(LENGTHS):
        ro, uo, To = _oracle_tube(fields[i], n_rot[i], tau[i], int(steps[i]), m)
        if dtype == "float64":
            assert np.abs(R[i] - ro).max() <= 1e-12 * np.abs(ro).max(), i
            assert np.abs(U[i] - uo[0]).max() <= 1e-12 * max(np.abs(uo).max(), 1.0), i
            assert np.abs(Tt[i] - To).max() <= 1e-12 * np.abs(To).max(), i
        else:
            for a_, b_ in ((R[i], ro), (U[i], uo[0]), (Tt[i], To)):
                assert np.abs(a_ - b_).max() <= 1e-5, i


def test_batched_equals_single_instance_runs(torch_cuda):
    from paper_1606_06107_amd import Batch
    announce("batched == single")
    lengths = [300, 1500, 40, 2500]
    n_rot, tau, steps, rho, u, T, fields = _mild_batch(2, lengths)
    b = Batch(lengths, n_rot, tau, steps, dtype=torch_cuda.float32).init(rho, u, T)
    b.step()
    fb = b.split(b.f[0])
    for i, L in enumerate(lengths):
        one = Batch([L], n_rot[i:i + 1], tau[i:i + 1], steps[i:i + 1], dtype=torch_cuda.float32)
        one.init(fields[i][0], fields[i][1][0], fields[i][2]).step()
        torch_cuda.cuda.synchronize()
        assert np.array_equal(one.f[0].cpu().numpy(), fb[i]), i


def test_batch_equals_per_step_kernel(torch_cuda):
    """The on-chip time loop and the per-step kernel agree (FP64)."""
    from paper_1606_06107_amd import Batch, Sim
    announce("batch vs per-step")
    L, n_rot, tau, steps = 800, 4.0, 0.8, 150
    rho, u, T = workloads.sod_tube(L, (4.0, 0.0, 4.0), (1.0, 0.0, 1.0))
    b = Batch([L], [n_rot], [tau], [steps], dtype=torch_cuda.float64).init(rho, u[0], T).step()
    sim = Sim((L,), bc=["open"], n_rot=n_rot, tau=tau, dtype=torch_cuda.float64).init(rho, u, T)
    sim.step(steps)
    r1 = b.moments()[0].cpu().numpy()
    r2 = sim.moments()[0].cpu().numpy()
    assert np.abs(r1 - r2).max() <= 1e-13 * np.abs(r2).max()


def test_every_tube_processed_and_ordered_queue(torch_cuda):
    from paper_1606_06107_amd import Batch
    announce("queue")
    rng = np.random.default_rng(5)
    lengths = rng.integers(4, 40, 3000)
    I = len(lengths)
    rho = np.ones(lengths.sum())
    b = Batch(lengths, np.full(I, 2.0), np.full(I, 0.8), rng.integers(0, 5, I),
              dtype=torch_cuda.float32).init(rho, np.zeros_like(rho), np.ones_like(rho))
    b.step()
    torch_cuda.cuda.synchronize()
    st = b.status.cpu().numpy()
    assert (st == 0).all()  # every tube written (initialised to -1)
    # uniform tubes stay uniform
    r = b.moments()[0].cpu().numpy()
    assert np.abs(r - 1.0).max() < 1e-6


def test_unstable_tube_flagged(torch_cuda):
    from paper_1606_06107_amd import Batch
    announce("status")
    lengths = [400, 400]
    f1 = workloads.sod_tube(400, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))   # classic Sod: diverges
    f2 = workloads.sod_tube(400, (1.0, 0.0, 1.0), (0.5, 0.0, 0.5))
    rho = np.concatenate([f1[0], f2[0]])
    u = np.concatenate([f1[1][0], f2[1][0]])
    T = np.concatenate([f1[2], f2[2]])
    b = Batch(lengths, [4.0, 4.0], [0.8, 0.8], [300, 300], dtype=torch_cuda.float32).init(rho, u, T)
    b.step()
    torch_cuda.cuda.synchronize()
    st = b.status.cpu().numpy()
    assert st[0] in (1, 2) and st[1] == 0


def test_long_tubes_fail_at_the_same_step_as_on_chip(torch_cuda):
    """Forcing 256-node chunks turns both tubes into multi-chunk, multi-pass
    work-queue tubes: the diverging one stops at the same step with the same
    status as in the whole-tube on-chip run, and the stable one ends with the
    same bits."""
    from paper_1606_06107_amd import Batch
    announce("long tube failure step")
    f1 = workloads.sod_tube(700, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))   # classic Sod: diverges
    f2 = workloads.sod_tube(700, (1.0, 0.0, 1.0), (0.5, 0.0, 0.5))
    rho = np.concatenate([f1[0], f2[0]])
    u = np.concatenate([f1[1][0], f2[1][0]])
    T = np.concatenate([f1[2], f2[2]])
    runs = []
    for chunk, sup in ((0, 0), (256, 8), (448, 24)):
        b = Batch([700, 700], [4.0, 4.0], [0.8, 0.8], [300, 300], dtype=torch_cuda.float32, chunk=chunk,
                  superstep=sup).init(rho, u, T)
        b.step()
        torch_cuda.cuda.synchronize()
        runs.append((b.status.cpu().numpy(), b.steps_done.cpu().numpy(), b.split(b.f[0])[1]))
    (st0, done0, f0), rest = runs[0], runs[1:]
    assert st0[0] in (1, 2) and st0[1] == 0 and 0 < done0[0] < 300 and done0[1] == 300
    for st, done, f in rest:
        assert np.array_equal(st, st0) and np.array_equal(done, done0)
        assert np.array_equal(f, f0)


def test_index_order_mode_beyond_sort_capacity(torch_cuda):
    """More tubes than the schedule sorts (16384): every tube runs from the
    queue in index order, a long one walking its chunks on one workgroup."""
    from paper_1606_06107_amd import Batch
    announce("index-order mode")
    rng = np.random.default_rng(11)
    small = rng.integers(4, 12, 16400)
    L0, steps0 = 1500, 60
    lengths = np.concatenate([[L0], small])
    I = len(lengths)
    r0, u0, T0 = workloads.sod_tube(L0, (1.0, 0.0, 1.0), (0.5, 0.0, 0.6))
    rest = int(small.sum())
    rho = np.concatenate([r0, np.ones(rest)])
    u = np.concatenate([u0[0], np.zeros(rest)])
    T = np.concatenate([T0, np.ones(rest)])
    steps = np.concatenate([[steps0], rng.integers(0, 6, I - 1)])
    b = Batch(lengths, np.full(I, 2.0), np.full(I, 0.8), steps, dtype=torch_cuda.float32, chunk=512,
              superstep=16).init(rho, u, T)
    b.step()
    torch_cuda.cuda.synchronize()
    assert (b.status.cpu().numpy() == 0).all()
    assert np.array_equal(b.steps_done.cpu().numpy(), steps)
    R, U, TT = (b.split(x) for x in b.moments())
    ro, uo, To = _oracle_tube((r0, u0, T0), 2.0, 0.8, steps0)
    for a_, b_ in ((R[0], ro), (U[0], uo[0]), (TT[0], To)):
        assert np.abs(a_ - b_).max() <= 1e-5
    assert max(np.abs(R[i] - 1.0).max() for i in range(1, I, 997)) < 1e-6


def test_batch_substeps_equal_per_step_path_and_noalloc(torch_cuda):
    """The batch kernel's sub-stepped rotational advection equals the
    per-step path's (lbm_step with g_substeps) on a tube, and the
    no-allocation launch gives the same bits as the graph launch."""
    import torch
    from paper_1606_06107_amd import Batch, Sim
    announce("batch substeps == per-step substeps")
    L, steps, m = 700, 60, 4
    rho, u, T = workloads.sod_tube(L, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    sim = Sim((L,), bc=["open"], n_rot=4.0, tau=1.0, dtype=torch.float64, g_substeps=m).init(rho, u, T)
    sim.step(steps)
    r1, u1, T1, _ = sim.moments()
    outs = []
    for noalloc in (False, True):
        b = Batch([L], [4.0], [1.0], [steps], dtype=torch.float64, g_substeps=m).init(rho, u[0], T)
        (b.step_noalloc if noalloc else b.step)()
        r2, u2, T2 = b.moments()
        torch.cuda.synchronize()
        assert int(b.status.cpu()[0]) == 0
        outs.append(torch.stack([r2, u2, T2]).cpu().numpy())
        b.release()
    ref = np.stack([r1.cpu().numpy(), u1[0].cpu().numpy(), T1.cpu().numpy()])
    assert np.abs(outs[0] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dtype,chunk,superstep", [("float64", 256, 8), ("float32", 0, 0)])
def test_zero_step_tubes_are_left_alone(torch_cuda, dtype, chunk, superstep):
    """Tubes with nsteps = 0 among stepped ones, on chip and chunked: their
    populations bitwise unchanged, status 0 and 0 steps; the stepped tubes
    against the oracle, and bitwise equal to a call that steps every tube."""
    import torch
    from paper_1606_06107_amd import Batch
    announce(f"zero-step tubes {dtype} chunk={chunk}")
    n_rot, tau, steps, rho, u, T, fields = _mild_batch(11)
    zero = np.arange(len(LENGTHS)) % 3 == 1  # tubes 17, 255, 700, 2000 nodes
    part = np.where(zero, 0, steps)
    dt = getattr(torch_cuda, dtype)
    b = Batch(LENGTHS, n_rot, tau, part, dtype=dt, chunk=chunk, superstep=superstep).init(rho, u, T)
    full = Batch(LENGTHS, n_rot, tau, steps, dtype=dt, chunk=chunk, superstep=superstep).init(rho, u, T)
    f_init, g_init = b.f[0].clone(), b.g[0].clone()
    b.step()
    full.step()
    torch.cuda.synchronize()
    st, done = b.status.cpu().numpy(), b.steps_done.cpu().numpy()
    assert (st == 0).all()
    assert (done == part).all()
    off = b.offsets_h
    for i in range(len(LENGTHS)):
        sl = slice(int(off[i]), int(off[i + 1]))
        if zero[i]:
            assert torch.equal(b.f[0][:, sl], f_init[:, sl]) and torch.equal(b.g[0][:, sl], g_init[:, sl]), i
        else:
            assert torch.equal(b.f[0][:, sl], full.f[0][:, sl]) and torch.equal(b.g[0][:, sl], full.g[0][:, sl]), i
    R, U, Tt = (b.split(m) for m in b.moments())
    for i in np.flatnonzero(~zero):
        ro, uo, To = _oracle_tube(fields[i], n_rot[i], tau[i], int(steps[i]))
        tol = 1e-12 if dtype == "float64" else 1e-5
        scale = (np.abs(ro).max(), max(np.abs(uo).max(), 1.0), np.abs(To).max()) if dtype == "float64" else (1, 1, 1)
        for a_, b_, sc in ((R[i], ro, scale[0]), (U[i], uo[0], scale[1]), (Tt[i], To, scale[2])):
            assert np.abs(a_ - b_).max() <= tol * sc, i


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_launch_shapes_give_the_same_bits(torch_cuda, dtype):
    """The tubes of one batch advanced in the library's default shape and in
    each latency shape of the surrogate's fallback (small chunks, long
    passes; per-call chunk and superstep overrides): the same status, steps
    and populations, bitwise -- halos are recomputed with the same per-node
    arithmetic, and only nodes a full halo away from a chunk's cut are kept."""
    import torch
    from paper_1606_06107_amd import Batch
    from paper_1606_06107_amd.surrogate import LATENCY_SHAPES
    announce(f"launch shapes, same bits ({dtype})")
    n_rot, tau, steps, rho, u, T, _ = _mild_batch(12)
    dt = getattr(torch_cuda, dtype)
    b = Batch(LENGTHS, n_rot, tau, steps, dtype=dt)
    ref = None
    for shape in [(0, 0)] + list(LATENCY_SHAPES):
        b.init(rho, u, T)
        b.step(chunk=shape[0], superstep=shape[1])
        torch.cuda.synchronize()
        got = (b.status.cpu().numpy().copy(), b.steps_done.cpu().numpy().copy(),
               b.f[0].cpu().numpy().copy(), b.g[0].cpu().numpy().copy())
        assert (got[0] == 0).all() and np.array_equal(got[1], steps), shape
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3]), shape
    b.release()


def test_degenerate_calls(torch_cuda):
    """Zero steps change nothing (Sim.step(0); a batch whose tubes all have
    0 steps: status 0, 0 steps done, populations bitwise unchanged), and the
    shortest tube the batch accepts (4 nodes) matches the oracle."""
    import torch
    from paper_1606_06107_amd import Batch, Sim
    from gpu_helpers import smooth_fields
    announce("degenerate calls")
    fields = smooth_fields((20, 12), 3)
    sim = Sim((20, 12), n_rot=2.0, tau=0.8, dtype=torch.float32).init(*fields)
    sim.step(3)
    f0, g0 = (t.clone() for t in sim.populations())
    t0 = sim.t
    sim.step(0)
    f1, g1 = sim.populations()
    assert sim.t == t0
    assert torch.equal(f0, f1) and torch.equal(g0, g1)

    lengths = [4, 9, 300]
    n_rot, tau, _, rho, u, T, _ = _mild_batch(7, lengths)
    b = Batch(lengths, n_rot, tau, np.zeros(3, dtype=np.int64), dtype=torch.float64).init(rho, u, T)
    fb, gb = b.f[0].clone(), b.g[0].clone()
    b.step()
    torch.cuda.synchronize()
    assert (b.status.cpu().numpy() == 0).all() and (b.steps_done.cpu().numpy() == 0).all()
    assert torch.equal(b.f[0], fb) and torch.equal(b.g[0], gb)

    n_rot, tau, _, rho, u, T, fl = _mild_batch(8, [4])
    b = Batch([4], n_rot, tau, [30], dtype=torch.float64).init(rho, u, T).step()
    want = _oracle_tube(fl[0], float(n_rot[0]), float(tau[0]), 30)
    got = [t.cpu().numpy() for t in b.moments()]
    assert (b.status.cpu().numpy() == 0).all()
    for k in range(3):
        assert np.abs(got[k] - np.asarray(want[k]).reshape(-1)).max() <= 1e-12 * max(1.0, np.abs(want[k]).max())
