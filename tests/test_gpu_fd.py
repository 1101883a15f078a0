"""GPU parity of the finite-difference update (lbm_set_fd: Sec. V A written
for the translational populations as well) against the oracle's FD mode,
through the C ABI."""
import numpy as np
import pytest

from gpu_helpers import abs_err, announce, field_err, gpu_run, oracle_run, rel_err, smooth_fields

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _check(g, o, dtype):
    for k in ("rho", "u", "T"):
        e = field_err(k, g[k], o[k], o["T"]) if dtype == "float64" else abs_err(g[k], o[k])
        assert e <= (FP64_TOL if dtype == "float64" else FP32_TOL), (k, e)


@pytest.mark.parametrize("shape,bc", [((150,), ["open"]), ((97,), ["periodic"]),
                                      ((40, 24), ["periodic", "periodic"]), ((70, 19), ["open", "periodic"]),
                                      ((130, 9), ["periodic", "open"]), ((71, 6), ["periodic", "periodic"])])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_fd_vs_oracle(torch_cuda, shape, bc, dtype):
    """12 steps at Courant factor 0.15 from smooth fields plus a
    non-equilibrium perturbation; ragged tiles (97, 150, 70x19, 130x9 with a
    ragged second tile and an open y axis, 71x6)."""
    announce(f"FD {dtype} {shape} {bc}")
    fields = smooth_fields(shape, 4)
    dt = getattr(torch_cuda, dtype)
    g = gpu_run(shape, bc, 3.0, 0.8, dt, fields, 12, perturb_seed=7, fd=0.15, chunks=[5, 7])
    o = oracle_run(shape, bc, 3.0, 0.8, fields, 12, perturb_seed=7, fd=0.15)
    _check(g, o, dtype)
    if dtype == "float64":
        assert rel_err(g["f"], o["f"]) <= FP64_TOL and rel_err(g["g"], o["g"]) <= FP64_TOL
        assert rel_err(g["tot"], o["tot"]) <= FP64_TOL


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_fd_d2q37_vs_oracle(torch_cuda, orc, dtype):
    """The FD update on the D2Q37 lattice (populations matched by velocity)."""
    import torch

    import workloads
    from gpu_helpers import slot_permutation
    from paper_1606_06107_amd import Sim, lattice_info
    announce(f"FD D2Q37 {dtype}")
    shape, bc = (36, 20), ["periodic", "open"]
    _, _, _, c_lib = lattice_info("D2Q37")
    c_orc, _, _ = orc.lattice(orc.D2Q37)
    perm = slot_permutation(c_lib, c_orc)
    fields = smooth_fields(shape, 9)
    N = shape[0] * shape[1]
    G = orc.Grid(orc.D2Q37, shape, bc=[orc.PERIODIC, orc.OPEN], n_rot=2.0, tau=0.9, fd_courant=0.12)
    f_o, g_o = G.init_eq(*fields)
    f_o *= workloads.nonequilibrium_perturbation((37, N), 31)
    sim = Sim(shape, bc=bc, n_rot=2.0, tau=0.9, dtype=getattr(torch_cuda, dtype), lattice="D2Q37")
    sim.init_populations(torch.as_tensor(f_o[perm]), torch.as_tensor(g_o)).set_fd(0.12)
    sim.step(10)
    rho, u, T, tot = (x.cpu().numpy() for x in sim.moments())
    G.step(f_o, g_o, 10)
    ro, uo, To, toto = G.moments(f_o, g_o)
    _check({"rho": rho, "u": u, "T": T}, {"rho": ro, "u": uo, "T": To}, dtype)
    if dtype == "float64":
        f = sim.populations()[0].double().cpu().numpy()
        assert rel_err(f, f_o[perm]) <= FP64_TOL and rel_err(tot, toto) <= FP64_TOL


def test_fd_shock_tube_long_run(torch_cuda):
    """The 1-D shock tube (rho 4:1 at T = 1, n = 4, tau = 2/3, open ends) over
    1800 FD steps at Courant factor 0.1 (the time of 180 streaming steps),
    FP64: fields within 2e-11 of the oracle through the shock."""
    announce("FD tube 1000 x 1800")
    N = 1000
    x = (np.arange(N) + 0.5) / N
    fields = (np.where(x < 0.5, 4.0, 1.0), np.zeros((1, N)), np.ones(N))
    g = gpu_run((N,), ["open"], 4.0, 2.0 / 3.0, torch_cuda.float64, fields, 1800, fd=0.1)
    o = oracle_run((N,), ["open"], 4.0, 2.0 / 3.0, fields, 1800, fd=0.1)
    for k in ("rho", "u", "T"):
        assert field_err(k, g[k], o[k], o["T"]) <= 2e-11, k


def test_fd_rules(torch_cuda):
    from paper_1606_06107_amd import Sim
    from paper_1606_06107_amd._lib import LBM_EINVAL, LBM_EUNSUPPORTED, LbmError
    announce("FD rules")
    f2 = smooth_fields((32, 16), 1)
    sim = Sim((32, 16), tau=0.8).init(*f2)
    sim.set_fd(0.2)
    with pytest.raises(LbmError) as e:
        sim.set_inplace(True)  # the FD update ping-pongs
    assert e.value.status == LBM_EUNSUPPORTED
    sim.set_monitor(1, 4)
    with pytest.raises(LbmError) as e:
        sim.step(1)
    assert e.value.status == LBM_EUNSUPPORTED
    sim.set_monitor(0, 0)
    sim.step(2)
    with pytest.raises(LbmError) as e:
        sim.set_fd(0.1)  # after the first step
    assert e.value.status == LBM_EINVAL
    with pytest.raises(LbmError) as e:
        Sim((32, 16), tau=0.8).init(*f2).set_fd(1.5)
    assert e.value.status == LBM_EINVAL
    f3 = smooth_fields((8, 6, 5), 1)
    with pytest.raises(LbmError) as e:
        Sim((8, 6, 5), tau=0.8).init(*f3).set_fd(0.2)
    assert e.value.status == LBM_EUNSUPPORTED
