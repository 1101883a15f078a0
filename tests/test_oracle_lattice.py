"""Pins of the oracle's lattices against the quadrature conditions and the
paper's Tables I and II (Sec. IV)."""
import itertools
import math

import numpy as np
import pytest

from conftest import golden


def dfact(k):
    """(k-1)!! for even k: moment of order k of the unit Gaussian; 0 for odd k."""
    if k % 2:
        return 0.0
    return float(np.prod(np.arange(k - 1, 0, -2))) if k > 1 else 1.0


def quad(c, w, r, alpha):
    x = (r * c[:, :len(alpha)]).astype(np.float64)
    return float(np.sum(w * np.prod(x ** np.array(alpha), axis=1)))


def quad_scale(c, w, r, alpha):
    """sum |w x^alpha|: the size that rounding in quad() is relative to."""
    x = (r * c[:, :len(alpha)]).astype(np.float64)
    return float(np.sum(np.abs(w * np.prod(x ** np.array(alpha), axis=1))))


def test_d1q7_gauss_moments_degree9(orc):
    c, w, r = orc.lattice(orc.D1Q7)
    assert len(w) == 7
    for k in range(10):
        assert quad(c, w, r, (k,)) == pytest.approx(dfact(k), rel=1e-14, abs=1e-15)
    # degree 10 is not integrated exactly: r is the degree-9 root, not another
    assert abs(quad(c, w, r, (10,)) - 945.0) > 1.0


def test_d1q7_matches_table2(orc):
    c, w, r = orc.lattice(orc.D1Q7)
    assert r == pytest.approx(1.1969797752, rel=5e-9)
    rows = golden("table2_d1q7.txt")
    for k, absc, wt in rows:
        k, absc, wt = int(k), int(absc), float(wt)
        members = [i for i in range(7) if abs(c[i, 0]) == absc]
        assert len(members) == k
        for i in members:
            assert w[i] == pytest.approx(wt, rel=1e-8)


def test_rotational_lattice_shares_r(orc):
    eta, wr = orc.rot_lattice()
    r = orc.d1q7_r()
    assert np.allclose(eta, r * np.arange(-3, 4), rtol=0, atol=1e-15)
    assert wr.sum() == pytest.approx(1.0, abs=1e-15)


def test_sec6_time_formula(orc):
    # Sec. VI: t = step / (X r) = 180 / (1000 r) = 0.1504
    assert round(180 / (1000 * orc.d1q7_r()), 4) == 0.1504


@pytest.mark.parametrize("kind,D", [("D2Q49", 2), ("D3Q343", 3)])
def test_tensor_lattices(orc, kind, D):
    c, w, r = orc.lattice(getattr(orc, kind))
    assert len(w) == 7 ** D
    assert w.sum() == pytest.approx(1.0, abs=1e-14)
    # every per-axis exponent up to 9 is exact (product of 1-D rules)
    exps = [0, 1, 2, 3, 4, 5, 8, 9] if D == 2 else [0, 2, 3, 4, 9]
    for alpha in itertools.product(exps, repeat=D):
        want = math.prod(dfact(a) for a in alpha)
        assert quad(c, w, r, alpha) == pytest.approx(
            want, rel=1e-13, abs=1e-14 * quad_scale(c, w, r, alpha))


def test_d2q37_structure_and_moments(orc):
    c, w, r = orc.lattice(orc.D2Q37)
    assert len(w) == 37
    pts = {(int(a), int(b)) for a, b, _ in c}
    assert len(pts) == 37
    assert w.sum() == pytest.approx(1.0, abs=1e-14)
    # isotropic degree-9 exactness, including the c_x^4 c_y^4 condition the
    # weights were not solved from
    for a in range(10):
        for b in range(10 - a):
            assert quad(c, w, r, (a, b)) == pytest.approx(
                dfact(a) * dfact(b), rel=1e-12, abs=1e-14 * quad_scale(c, w, r, (a, b)))


def test_d2q37_matches_table1(orc):
    c, w, r = orc.lattice(orc.D2Q37)
    rows = golden("table1_d2q37.txt")
    for kp, members, p, q, wt in rows:
        members, p, q, wt = int(members), int(p), int(q), float(wt)
        idx = [i for i in range(37)
               if sorted((abs(c[i, 0]), abs(c[i, 1]))) == sorted((p, q))]
        assert len(idx) == members
        for i in idx:
            assert w[i] == pytest.approx(wt, rel=2e-7)
