"""lbm_batch_step_noalloc (the batched launch on the library's fixed device
scratch, for callers that cannot allocate) against lbm_batch_step on the
same tubes: bitwise equal populations, status and steps, on two calls in a
row, the second on a smaller batch."""
import numpy as np
import pytest

from gpu_helpers import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _tubes(n, seed, long_every):
    """Shock tubes of the batched recipe's states; every `long_every`-th tube
    is longer than one on-chip chunk, so both phases of the launch run."""
    rng = np.random.default_rng(seed)
    lengths = rng.integers(64, 1200, n)
    lengths[::long_every] = rng.integers(3000, 9000, len(lengths[::long_every]))
    gam = rng.uniform(1.2, 1.67, n)
    n_rot = 2.0 / (gam - 1.0) - 1.0
    tau = rng.uniform(0.6, 1.0, n)
    steps = rng.integers(0, 400, n)
    rho, u, T = [], [], []
    for L in lengths:
        x = (np.arange(L) + 0.5) / L
        left = x < 0.5
        rho.append(np.where(left, 1.0, 0.5))
        u.append(np.zeros(L))
        T.append(np.where(left, 1.0, 0.8))
    return lengths, n_rot, tau, steps, np.concatenate(rho), np.concatenate(u), np.concatenate(T)


def _run(torch, case, noalloc, dtype):
    from paper_1606_06107_amd import Batch
    lengths, n_rot, tau, steps, rho, u, T = case
    b = Batch(lengths, n_rot, tau, steps, dtype=dtype).init(rho, u, T)
    (b.step_noalloc if noalloc else b.step)()
    torch.cuda.synchronize()
    out = (b.f[0].cpu().numpy(), b.g[0].cpu().numpy(), b.status.cpu().numpy(), b.steps_done.cpu().numpy())
    b.release()
    return out


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_noalloc_batch_equals_batch_step(torch_cuda, dtype_name):
    dtype = getattr(torch_cuda, dtype_name)
    big = _tubes(300, 11, 25)
    small = _tubes(40, 12, 7)
    for name, case in (("300 tubes", big), ("40 tubes", small)):  # the second call is smaller
        announce(f"no-alloc batch {dtype_name} {name}")
        ref = _run(torch_cuda, case, False, dtype)
        got = _run(torch_cuda, case, True, dtype)
        assert (ref[2] >= 0).all()
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
