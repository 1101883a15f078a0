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


# ---------------------------------------------------------------------------
# Hand-built networks: every parameter zero except a few chosen ones, so the
# output follows from the network's written definition by hand arithmetic.
# They fix what a self-consistent mistake (kernel and reference written to
# the same wrong reading) would get wrong: the feature order p*4 + c, the
# normalisation, the conv tap orientation and its per-tube zero padding, the
# residual MLP and its GELU, the output order 3p + c and scale 0.1.
# ---------------------------------------------------------------------------
def _zero():
    return {name: np.zeros(shape) for name, shape in S.layout()}


def _fields(B, L, seed):
    rng = np.random.default_rng(seed)
    x = np.stack([0.5 + 0.4 * rng.uniform(size=(B, L)), 0.3 * rng.normal(size=(B, L)),
                  0.8 + 0.3 * rng.uniform(size=(B, L))])
    gamma = rng.uniform(1.1, 1.67, B)
    return x, gamma


MU = {0: 0.5, 1: 0.0, 2: 1.0, 3: 1.4}   # rho, u, T, gamma
SD = {0: 0.5, 1: 0.5, 2: 0.5, 3: 0.3}


def _feature(x, gamma, c, b, node):
    v = gamma[b] if c == 3 else x[c, b, node]
    return (v - MU[c]) / SD[c]


@pytest.mark.parametrize("p0,c0,p1,c1", [(2, 3, 1, 2), (0, 1, 3, 0), (3, 2, 0, 1), (1, 0, 2, 2)])
def test_feature_and_output_order(p0, c0, p1, c1):
    """Embedding row 0 reads feature p0*4 + c0 (field c0 of node 4t + p0);
    the head writes it to output 3*p1 + c1, i.e. field c1 of node 4t + p1,
    scaled by 0.1 on top of the input.  No other output changes."""
    B, L = 2, 32
    x, gamma = _fields(B, L, 5)
    d = _zero()
    d["We"][0, p0 * 4 + c0] = 1.0
    d["Wh"][3 * p1 + c1, 0] = 1.0
    y, _ = S.forward(d, x, gamma, rounded=False)
    want = x.copy()
    for b in range(B):
        for t in range(L // 4):
            want[c1, b, 4 * t + p1] += 0.1 * _feature(x, gamma, c0, b, 4 * t + p0)
    assert np.abs(y - want).max() < 1e-15


@pytest.mark.parametrize("k0", range(5))
def test_conv_tap_orientation_and_tube_padding(k0):
    """Block 0 with only tap k0 of channel 0 set: Hc[t] = H[t] + bc + H[t + k0 - 2],
    the neighbour taken from the same tube and zero beyond its ends; the head
    passes channel 0 to the rho output of each token's first node."""
    B, L = 2, 40
    T = L // 4
    x, gamma = _fields(B, L, 6)
    d = _zero()
    d["We"][0, 0] = 1.0          # channel 0 = normalised rho of node 4t
    d["kc0"][0, k0] = 1.0
    d["bc0"][0] = 0.25
    d["Wh"][0, 0] = 1.0
    y, _ = S.forward(d, x, gamma, rounded=False)
    s = k0 - 2
    for b in range(B):
        for t in range(T):
            h = _feature(x, gamma, 0, b, 4 * t) + 0.25
            if 0 <= t + s < T:
                h += _feature(x, gamma, 0, b, 4 * (t + s))
            assert y[0, b, 4 * t] == pytest.approx(x[0, b, 4 * t] + 0.1 * h, abs=1e-15)


def _golden_gelu():
    from conftest import golden
    return [(float(z), float(v)) for z, v in golden("gelu_tanh.txt")]


def test_residual_mlp_gelu():
    """Block 0's MLP on channel 0 only: Z1 = 2 Hc + b1 (W1[0,0] = 2, b1 = 0.5),
    H' = Hc + 3 gelu(Z1) + b2 (W2[0,0] = 3, b2 = -0.125).  Hc is set per token
    by the input so that Z1 runs through the tabulated GELU points."""
    pts = _golden_gelu()
    B, L = 1, 4 * len(pts)
    x, gamma = _fields(B, L, 7)
    # rho of node 4t chosen so that Z1 = 2 ((rho - 0.5)/0.5) + 0.5 = z_t
    for t, (z, _) in enumerate(pts):
        x[0, 0, 4 * t] = 0.5 + 0.5 * (z - 0.5) / 2.0
    d = _zero()
    d["We"][0, 0] = 1.0
    d["W10"][0, 0] = 2.0
    d["b10"][0] = 0.5
    d["W20"][0, 0] = 3.0
    d["b20"][0] = -0.125
    d["Wh"][0, 0] = 1.0
    y, _ = S.forward(d, x, gamma, rounded=False)
    for t, (z, gz) in enumerate(pts):
        hc = (z - 0.5) / 2.0
        want = x[0, 0, 4 * t] + 0.1 * (hc + 3.0 * gz - 0.125)
        assert y[0, 0, 4 * t] == pytest.approx(want, abs=1e-14), z


def test_bf16_points_on_representable_values():
    """With every weight and input feature exactly representable in BF16,
    rounding acts at two points here: the GELU output and the head's input
    H4 (matrix-product operands).  rounded=True then gives the hand value
    with gelu(z) and H4 replaced by their BF16 roundings."""
    pts = _golden_gelu()
    B, L = 1, 4 * len(pts)
    x, gamma = _fields(B, L, 8)
    gamma[:] = 1.4 + 0.3 * 0.5          # feature 0.5
    x[1] = 0.0
    x[2] = 1.0
    for t, (z, _) in enumerate(pts):
        x[0, 0, 4 * t] = 0.5 + 0.5 * (z - 0.5) / 2.0  # features (z - 0.5)/2: short binary fractions
    d = _zero()
    d["We"][0, 0] = 1.0
    d["W10"][0, 0] = 2.0
    d["b10"][0] = 0.5
    d["W20"][0, 0] = 3.0
    d["Wh"][0, 0] = 1.0
    y, _ = S.forward(d, x, gamma, rounded=True)
    for t, (z, gz) in enumerate(pts):
        hc = (z - 0.5) / 2.0
        want = x[0, 0, 4 * t] + 0.1 * S.bf16(hc + 3.0 * S.bf16(gz))
        assert y[0, 0, 4 * t] == pytest.approx(want, abs=1e-14), z
