"""Pins of the oracle's equilibria (Sec. IV) against closed-form Gaussian
moments (Sec. II moment integrals, and the moment list of the Appendix)."""
import itertools
import math

import numpy as np
import pytest


def gauss_raw_moment(k, mu, var):
    """E[x^k] for x ~ N(mu, var), by the binomial expansion with central
    moments (j-1)!! var^(j/2)."""
    s = 0.0
    for j in range(0, k + 1, 2):
        cm = float(np.prod(np.arange(j - 1, 0, -2))) if j > 1 else 1.0
        s += math.comb(k, j) * mu ** (k - j) * cm * var ** (j // 2)
    return s


CASES = [(1.3, (0.2, -0.1, 0.15), 0.9), (0.7, (-0.3, 0.25, 0.1), 1.2),
         (2.0, (0.05, 0.0, -0.2), 1.0), (1.0, (0.0, 0.0, 0.0), 0.75)]


@pytest.mark.parametrize("kind,D", [("D1Q7", 1), ("D2Q49", 2), ("D2Q37", 2), ("D3Q343", 3)])
@pytest.mark.parametrize("case", CASES)
def test_feq_reproduces_maxwellian_moments_to_order4(orc, kind, D, case):
    rho, u, T = case
    u = np.array(u[:D])
    c, w, r = orc.lattice(getattr(orc, kind))
    fe = orc.feq(getattr(orc, kind), rho, u, T)
    xi = r * c[:, :D].astype(np.float64)
    for order in range(5):
        for alpha in itertools.product(range(order + 1), repeat=D):
            if sum(alpha) != order:
                continue
            got = float(np.sum(fe * np.prod(xi ** np.array(alpha), axis=1)))
            want = rho * math.prod(gauss_raw_moment(a, u[d], T) for d, a in enumerate(alpha))
            assert got == pytest.approx(want, rel=1e-12, abs=1e-12), (alpha, got, want)


def test_appendix_moment_list_2d(orc):
    """The Appendix moment list with P = rho T, e_t = D T / 2 (D = 2): second
    and third velocity moments and the contracted energy fluxes.  The energy
    flux carries the pressure work P u (the Gaussian integral), which the
    printed entry for sum g^eq xi^2 xi / 2 leaves out."""
    rho, u, T = 1.1, np.array([0.3, -0.2]), 0.95
    D, P, et = 2, rho * T, T
    c, w, r = orc.lattice(orc.D2Q49)
    fe = orc.feq(orc.D2Q49, rho, u, T)
    xi = r * c[:, :2].astype(np.float64)
    I = np.eye(2)
    M2 = np.einsum("i,ia,ib->ab", fe, xi, xi)
    assert np.allclose(M2, rho * np.outer(u, u) + P * I, atol=1e-13)
    M3 = np.einsum("i,ia,ib,ic->abc", fe, xi, xi, xi)
    want3 = rho * np.einsum("a,b,c->abc", u, u, u) + P * (
        np.einsum("a,bc->abc", u, I) + np.einsum("b,ac->abc", u, I) + np.einsum("c,ab->abc", u, I))
    assert np.allclose(M3, want3, atol=1e-13)
    xi2 = (xi ** 2).sum(1)
    E1 = np.einsum("i,i,ia->a", fe, 0.5 * xi2, xi)
    assert np.allclose(E1, rho * (0.5 * u @ u + et) * u + P * u, atol=1e-13)
    E2 = np.einsum("i,i,ia,ib->ab", fe, 0.5 * xi2, xi, xi)
    want = P * (2.0 / D * et + 0.5 * u @ u + et) * I + (2 * P + 0.5 * rho * u @ u + rho * et) * np.outer(u, u)
    assert np.allclose(E2, want, atol=1e-13)


@pytest.mark.parametrize("T", [0.6, 0.8, 1.0, 1.3, 2.0])
def test_geq_moments(orc, T):
    eta, _ = orc.rot_lattice()
    ge = orc.geq(T)
    assert ge.sum() == pytest.approx(1.0, abs=1e-15)
    assert (ge * eta).sum() == pytest.approx(0.0, abs=1e-15)
    assert (ge * eta ** 2).sum() == pytest.approx(T, rel=1e-14)
    assert (ge * eta ** 3).sum() == pytest.approx(0.0, abs=1e-14)
    assert (ge * eta ** 4).sum() == pytest.approx(3 * T * T, rel=1e-14)


def test_equilibria_at_rest_are_weights(orc):
    c, w, r = orc.lattice(orc.D2Q49)
    assert np.allclose(orc.feq(orc.D2Q49, 1.0, [0.0, 0.0], 1.0), w, rtol=0, atol=1e-16)
    eta, wr = orc.rot_lattice()
    assert np.allclose(orc.geq(1.0), wr, rtol=0, atol=1e-16)


@pytest.mark.parametrize("kind,D", [(1, 1), (2, 2), (3, 3)])
@pytest.mark.parametrize("n_rot", [0.0, 2.0, 11.0 / 3.0, 19.0])
def test_heat_capacity_ratio_from_discrete_equilibria(orc, kind, D, n_rot):
    """gamma = (D+n+2)/(D+n) (Sec. III) as a property of the discrete
    equilibria, not of the formula: the internal energy per unit mass of the
    equilibrium state at rest, (sum_i f^eq xi_i^2/2 + rho (n/2) sum_j g^eq
    eta_j^2) / rho, differentiated in T gives c_v; the pressure from the
    second moment, sum_i f^eq xi_x^2, gives R = p / (rho T); gamma = 1 + R/c_v."""
    c, w, r = orc.lattice(kind)
    xi = r * c[:, :D].astype(np.float64)
    eta, _ = orc.rot_lattice()
    rho, T, h = 1.3, 0.9, 1e-4

    def e_int(Tv):
        f = orc.feq(kind, rho, [0.0] * D, Tv)
        g = orc.geq(Tv)
        return ((f * (xi ** 2).sum(1)).sum() / 2 + rho * (n_rot / 2) * (g * eta ** 2).sum()) / rho

    cv = (e_int(T + h) - e_int(T - h)) / (2 * h)
    p = (orc.feq(kind, rho, [0.0] * D, T) * xi[:, 0] ** 2).sum()
    gamma = 1.0 + (p / (rho * T)) / cv
    assert gamma == pytest.approx((D + n_rot + 2) / (D + n_rot), rel=1e-9)
