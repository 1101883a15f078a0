"""Pins of the FP64 surrogate reference: gradients against central finite
differences of its own loss, and the adjoint identity of the convolution."""
import numpy as np
import pytest

from oracle import surrogate_ref as S


def _problem(seed=0, B=2, L=128):
    rng = np.random.default_rng(seed)
    x = np.stack([0.5 + 0.4 * rng.uniform(size=(B, L)), 0.3 * rng.normal(size=(B, L)),
                  0.8 + 0.3 * rng.uniform(size=(B, L))])
    target = x + 0.01 * rng.normal(size=x.shape)
    gamma = rng.uniform(1.1, 1.67, B)
    p = S.init_params(seed)
    # larger output weights so every layer matters in the check
    d = S.unpack(p)
    d["Wh"] = rng.normal(0, 0.2, d["Wh"].shape)
    for b in range(S.NB):
        d[f"W2{b}"] *= 5.0
    return S.pack(d), x, gamma, target


def test_parameter_count():
    assert S.NPARAMS == 69708
    p = S.init_params(0)
    assert np.array_equal(S.pack(S.unpack(p)), p)


def test_conv_adjoint():
    rng = np.random.default_rng(1)
    T = 16
    H = rng.normal(size=(3 * T, S.C))
    D = rng.normal(size=(3 * T, S.C))
    kc = rng.normal(size=(S.C, S.TAPS))
    assert np.sum(S._conv(H, kc, T) * D) == pytest.approx(np.sum(H * S._conv_t(D, kc, T)), rel=1e-12)


def test_gradients_match_finite_differences():
    p, x, gamma, target = _problem()
    loss, g, _ = S.loss_and_grads(S.unpack(p), x, gamma, target, rounded=False)
    gvec = S.pack(g)
    rng = np.random.default_rng(3)
    # every tensor gets at least a few probes
    offsets, o = [], 0
    for name, shape in S.layout():
        n = int(np.prod(shape))
        offsets += list(o + rng.choice(n, size=min(n, 6), replace=False))
        o += n
    h = 1e-6
    for i in offsets:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp = S.loss_and_grads(S.unpack(pp), x, gamma, target, rounded=False)[0]
        lm = S.loss_and_grads(S.unpack(pm), x, gamma, target, rounded=False)[0]
        fd = (lp - lm) / (2 * h)
        # central differences with h = 1e-6 carry ~1e-9 of rounding noise
        assert gvec[i] == pytest.approx(fd, rel=1e-5, abs=2e-9), i


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.0e-40])
    want = np.array([1.0, 1.0, 1.0 + 4 * 2 ** -8, 1.0, -2.5, 0.0])
    got = S.bf16(vals)
    assert got[0] == want[0] and got[1] == want[1] and got[2] == want[2] and got[3] == want[3]
    assert got[4] == want[4]


def test_identity_network_reproduces_input():
    p = S.init_params(0)
    d = S.unpack(p)
    d["Wh"][:] = 0.0
    d["bh"][:] = 0.0
    _, x, gamma, _ = _problem()
    y, _ = S.forward(d, x, gamma)
    assert np.array_equal(y, x)
