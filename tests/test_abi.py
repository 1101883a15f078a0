"""CPU-only checks of the C ABI (no kernel launches): the library loads and
exports every function include/lbm.h declares, host-side validation returns
the documented status codes, and the library's lattice constants agree with
the oracle's independent derivation."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1606_06107_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblbmx.so not built")
    return _lib


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("lbm_init", "lbm_step", "lbm_moments", "lbm_batch_step", "lbm_sur_forward",
              "lbm_sur_backward", "lbm_sur_adam", "lbm_sur_check", "lbm_sur_lift"):
        assert n in names


def test_every_declared_symbol_is_exported_and_bound(lib):
    L = lib.load()
    for name in _declared():
        assert hasattr(L, name), name
        assert name in lib.SIGNATURES, f"{name} has no ctypes signature"


def _desc(lib, **kw):
    d = lib.LbmDesc()
    d.abi_version = lib.LBM_ABI_VERSION
    d.dim, d.lattice, d.dtype = 2, lib.LBM_D2Q49, lib.LBM_F32
    d.n[0], d.n[1], d.n[2] = 64, 32, 1
    d.bc[0] = d.bc[1] = d.bc[2] = lib.LBM_BC_PERIODIC
    d.n_rot, d.tau = 3.0, 0.8
    for k in range(2):
        d.f[k] = 0x1000 * (k + 1)
        d.g[k] = 0x10000 * (k + 1)
    d.workspace = 0x100000
    for k, v in kw.items():
        if k == "n":
            for a in range(3):
                d.n[a] = v[a]
        else:
            setattr(d, k, v)
    return d


@pytest.mark.parametrize("bad,why", [
    (dict(abi_version=99), "abi_version"),
    (dict(dim=4), "dim"),
    (dict(lattice=1), "lattice"),
    (dict(dtype=7), "dtype"),
    (dict(n=(2, 32, 1)), "periodic"),
    (dict(n=(64, 32, 2)), "unused axis"),
    (dict(tau=0.5), "tau"),
    (dict(n_rot=-1.0), "n_rot"),
    (dict(workspace=0x100001), "aligned"),
])
def test_init_rejects_invalid_descriptors(lib, bad, why):
    L = lib.load()
    d = _desc(lib, **bad)
    h = ctypes.c_void_p()
    one = ctypes.c_void_p(0x2000)
    st = L.lbm_init(ctypes.byref(d), one, one, one, None, ctypes.byref(h))
    assert st == lib.LBM_EINVAL
    assert why in L.lbm_last_error().decode()
    assert not h.value


def test_null_fields_and_handles(lib):
    L = lib.load()
    d = _desc(lib)
    h = ctypes.c_void_p()
    assert L.lbm_init(ctypes.byref(d), None, None, None, None, ctypes.byref(h)) == lib.LBM_EINVAL
    assert L.lbm_step(None, 1) == lib.LBM_EINVAL
    assert L.lbm_set_blocked(None, 1) == lib.LBM_EINVAL
    assert L.lbm_set_inplace(None, 1) == lib.LBM_EINVAL
    assert L.lbm_moments(None, None, None, None, None) == lib.LBM_EINVAL
    assert L.lbm_destroy(None) == lib.LBM_OK


def test_valid_descriptor_without_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    L = lib.load()
    d = _desc(lib)
    h = ctypes.c_void_p()
    one = ctypes.c_void_p(0x2000)
    assert L.lbm_init(ctypes.byref(d), one, one, one, None, ctypes.byref(h)) == lib.LBM_EDEVICE


def test_workspace_sizes(lib):
    L = lib.load()
    d = _desc(lib, n=(1024, 1024, 1))
    nb = L.lbm_workspace_bytes(ctypes.byref(d))
    assert nb % 256 == 0 and nb >= (1024 * 1024 // 64) * 4 * 8  # one FP64 row per smallest tile
    bd = lib.LbmBatchDesc()
    bd.abi_version, bd.num_instances = lib.LBM_ABI_VERSION, 4096
    assert L.lbm_batch_workspace_bytes(ctypes.byref(bd)) >= 4096 * 4
    assert L.lbm_sur_bf16_bytes() == 2 * (1024 + 4 * 49152 + 32 * 64 + 64 * 16)
    sd = lib.LbmSurDesc()
    sd.abi_version, sd.batch, sd.length = lib.LBM_ABI_VERSION, 2, 256
    assert L.lbm_sur_workspace_bytes(ctypes.byref(sd)) > 2 * 64 * 64 * 4 * 9


def test_batch_validation(lib):
    L = lib.load()
    bd = lib.LbmBatchDesc()
    bd.abi_version = lib.LBM_ABI_VERSION
    bd.dtype, bd.num_instances, bd.total_nodes = lib.LBM_F32, 4, 100
    assert L.lbm_batch_step(ctypes.byref(bd), None) == lib.LBM_EINVAL  # NULL arrays
    bd.offsets = bd.n_rot = bd.tau = bd.nsteps = bd.status = bd.workspace = 0x1000
    bd.f[0], bd.f[1], bd.g[0], bd.g[1] = 0x2000, 0x3000, 0x4000, 0x5000
    bd.block = 300
    assert L.lbm_batch_step(ctypes.byref(bd), None) == lib.LBM_EINVAL
    assert "block" in L.lbm_last_error().decode()
    bd.block, bd.superstep = 0, 200
    assert L.lbm_batch_step(ctypes.byref(bd), None) == lib.LBM_EINVAL


@pytest.mark.parametrize("dim,kind", [(1, "D1Q7"), (2, "D2Q49"), (3, "D3Q343"), ("D2Q37", "D2Q37")])
def test_library_lattice_agrees_with_oracle(lib, orc, dim, kind):
    from paper_1606_06107_amd import lattice_info
    Q, r, w, c = lattice_info(dim)
    co, wo, ro = orc.lattice(getattr(orc, kind))
    assert Q == len(wo)
    # 50-digit derivation (library) vs FP64 bisection on the moment residual
    # (oracle): agreement to the oracle's root-finding accuracy
    assert r == pytest.approx(ro, rel=1e-14)
    if kind == "D2Q37":  # same velocity set, the library's slot order (slot Q-1-s holds -c_s)
        index = {tuple(int(v) for v in row[:2]): k for k, row in enumerate(co)}
        perm = np.array([index[tuple(int(v) for v in row[:2])] for row in c])
        assert sorted(perm) == list(range(Q))
        assert np.array_equal(c[::-1], -c)
        co, wo = co[perm], wo[perm]
    assert np.array_equal(c, co)
    assert np.allclose(w, wo, rtol=1e-13, atol=0)


def test_surrogate_parameter_layout_matches_reference(lib):
    from oracle import surrogate_ref as S
    from paper_1606_06107_amd import surrogate
    assert S.NPARAMS == lib.LBM_SUR_NPARAMS == surrogate.NPARAMS


def test_batch_release_rejects_null(lib):
    L = lib.load()
    assert L.lbm_batch_release(None) == lib.LBM_EINVAL
    assert L.lbm_prepare(None, 5) == lib.LBM_EINVAL


def test_batch_noalloc_rejects_oversized_batch(lib):
    """The fixed scratch holds 8 MiB; a batch needing more is refused before
    any device work."""
    L = lib.load()
    d = lib.LbmBatchDesc()
    d.abi_version = lib.LBM_ABI_VERSION
    d.dtype = lib.LBM_F32
    d.num_instances = 1000
    d.total_nodes = (1 << 31) - 1
    assert L.lbm_batch_workspace_bytes(ctypes.byref(d)) > 8 << 20
    assert L.lbm_batch_step_noalloc(ctypes.byref(d), None) == lib.LBM_EINVAL
    assert b"scratch" in L.lbm_last_error()
    assert L.lbm_batch_step_noalloc(None, None) == lib.LBM_EINVAL


def test_surrogate_lift_validates_the_fallback_batch(lib):
    """lbm_sur_lift refuses a fallback batch of the wrong type or size before
    any device work (the writes go to the batch's buffers)."""
    L = lib.load()
    s = lib.LbmSurDesc()
    s.abi_version = lib.LBM_ABI_VERSION
    s.batch, s.length = 4, 256
    b = lib.LbmBatchDesc()
    b.abi_version = lib.LBM_ABI_VERSION
    b.dtype = lib.LBM_F64
    b.num_instances, b.total_nodes = 4, 4 * 256
    for k in range(2):
        b.f[k] = b.g[k] = 0x1000 * (k + 1)
    b.nsteps = b.offsets = 0x2000
    x = acc = valid = ctypes.c_void_p(0x3000)
    assert L.lbm_sur_lift(ctypes.byref(s), x, acc, valid, ctypes.byref(b), 16, None) == lib.LBM_EINVAL
    assert b"FP32" in L.lbm_last_error()
    b.dtype = lib.LBM_F32
    b.total_nodes = 4 * 255
    assert L.lbm_sur_lift(ctypes.byref(s), x, acc, valid, ctypes.byref(b), 16, None) == lib.LBM_EINVAL
    b.total_nodes, b.num_instances = 4 * 256, 3
    assert L.lbm_sur_lift(ctypes.byref(s), x, acc, valid, ctypes.byref(b), 16, None) == lib.LBM_EINVAL
    assert L.lbm_sur_lift(ctypes.byref(s), x, acc, valid, None, 16, None) == lib.LBM_EINVAL
    assert L.lbm_sur_check(ctypes.byref(s), x, x, x, 1e-3, 1e-3, 1e-3, -1.0, acc, None) == lib.LBM_EINVAL


def test_surrogate_rollout_refuses_a_mismatched_batch():
    """The Python front end checks the fallback batch's type and tube
    lengths before the library is asked (no device work)."""
    torch = pytest.importorskip("torch")
    from paper_1606_06107_amd.surrogate import Surrogate

    class FakeBatch:
        dtype = torch.float64
        I = 2
        offsets_h = np.array([0, 256, 512])

    sur = Surrogate.__new__(Surrogate)
    sur.B, sur.L = 2, 256
    with pytest.raises(ValueError):
        sur.check_fallback(FakeBatch())
    FakeBatch.dtype = torch.float32
    sur.check_fallback(FakeBatch())
    FakeBatch.offsets_h = np.array([0, 128, 512])
    with pytest.raises(ValueError):
        sur.check_fallback(FakeBatch())


def test_stream_copy_rejects_unaligned(lib):
    L = lib.load()
    assert L.lbm_stream_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 24, None) == lib.LBM_EINVAL
    assert L.lbm_stream_copy(ctypes.c_void_p(0x1008), ctypes.c_void_p(0x2000), 32, None) == lib.LBM_EINVAL
    assert L.lbm_stream_copy(None, ctypes.c_void_p(0x2000), 32, None) == lib.LBM_EINVAL
    assert L.lbm_stream_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 0, None) == lib.LBM_OK


def test_pattern_probe_rejects_bad_arguments(lib):
    L = lib.load()
    a, b, c, d = (ctypes.c_void_p(v) for v in (0x1000, 0x2000, 0x3000, 0x4000))
    assert L.lbm_pattern_probe(0, 0, a, a, c, d, 64, 64, None) == lib.LBM_EINVAL   # ping-pong needs two f
    assert L.lbm_pattern_probe(1, 0, a, b, c, d, 64, 64, None) == lib.LBM_EINVAL   # in place needs one f
    assert L.lbm_pattern_probe(2, 0, a, a, c, c, 64, 64, None) == lib.LBM_EINVAL   # g distinct
    assert L.lbm_pattern_probe(6, 0, a, b, c, d, 64, 64, None) == lib.LBM_EINVAL
    assert L.lbm_pattern_probe(3, 0, a, b, c, d, 96, 64, None) == lib.LBM_EINVAL  # blocked: nx % 64
    assert L.lbm_pattern_probe(4, 0, a, b, c, d, 64, 64, None) == lib.LBM_EINVAL
    assert L.lbm_pattern_probe(0, 4, a, b, c, d, 64, 64, None) == lib.LBM_EINVAL
    assert L.lbm_pattern_probe(0, 0, a, b, c, d, 3, 64, None) == lib.LBM_EINVAL
    assert L.lbm_pattern_probe(0, 0, a, b, c, d, 64, 70000, None) == lib.LBM_EINVAL
    assert L.lbm_pattern_probe(0, 0, None, b, c, d, 64, 64, None) == lib.LBM_EINVAL


def test_pattern_probe_3d_rejects_bad_arguments(lib):
    L = lib.load()
    a, b, c, d = (ctypes.c_void_p(v) for v in (0x1000, 0x2000, 0x3000, 0x4000))
    assert L.lbm_pattern_probe_3d(0, a, a, c, d, 64, 8, 8, None) == lib.LBM_EINVAL    # f distinct
    assert L.lbm_pattern_probe_3d(0, a, b, c, c, 64, 8, 8, None) == lib.LBM_EINVAL    # g distinct
    assert L.lbm_pattern_probe_3d(3, a, b, c, d, 64, 8, 8, None) == lib.LBM_EINVAL
    assert L.lbm_pattern_probe_3d(0, a, b, c, d, 96, 8, 8, None) == lib.LBM_EINVAL    # n0 % 64
    assert L.lbm_pattern_probe_3d(0, a, b, c, d, 64, 3, 8, None) == lib.LBM_EINVAL
    assert L.lbm_pattern_probe_3d(0, a, b, c, d, 1024, 1024, 1024, None) == lib.LBM_EINVAL  # 2^32 bytes
    assert L.lbm_pattern_probe_3d(0, None, b, c, d, 64, 8, 8, None) == lib.LBM_EINVAL
