"""Pins of the exact Riemann solver (the Sod analytical solution of Sec. VI)
against a textbook table and the jump conditions."""
import math

import numpy as np
import pytest

from conftest import golden
from oracle import riemann


def test_toro_test1_star_state():
    want = {k: float(v) for k, v in golden("sod_toro_test1.txt")}
    p, u, rl, rr = riemann.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    assert p == pytest.approx(want["p_star"], abs=1e-5)
    assert u == pytest.approx(want["u_star"], abs=1e-5)
    assert rl == pytest.approx(want["rho_star_L"], abs=1e-5)
    assert rr == pytest.approx(want["rho_star_R"], abs=1e-5)


@pytest.mark.parametrize("left,right,gamma", [((4, 0, 4), (1, 0, 1), 1.4),
                                              ((1, 0, 1), (0.125, 0, 0.1), 1.4),
                                              ((1, 0, 1), (0.3, 0, 0.02), 1.25),
                                              ((1, 0.2, 1), (0.5, -0.1, 0.4), 5 / 3)])
def test_jump_conditions(left, right, gamma):
    p, u, rl, rr = riemann.star_state(left, right, gamma)
    # right-going shock (p* > p_R in all cases here): Rankine-Hugoniot
    rR, uR, pR = right
    assert p > pR
    S = riemann.wave_speeds(left, right, gamma)[1]
    m1 = rR * (uR - S)
    m2 = rr * (u - S)
    assert m1 == pytest.approx(m2, rel=1e-10)
    assert rR * (uR - S) ** 2 + pR == pytest.approx(rr * (u - S) ** 2 + p, rel=1e-10)
    h1 = gamma / (gamma - 1) * pR / rR + 0.5 * (uR - S) ** 2
    h2 = gamma / (gamma - 1) * p / rr + 0.5 * (u - S) ** 2
    assert h1 == pytest.approx(h2, rel=1e-10)
    # left rarefaction (p* < p_L): isentropic, Riemann invariant u + 2c/(g-1)
    rL, uL, pL = left
    assert p < pL
    assert pL / rL ** gamma == pytest.approx(p / rl ** gamma, rel=1e-10)
    cL = math.sqrt(gamma * pL / rL)
    cs = math.sqrt(gamma * p / rl)
    assert uL + 2 * cL / (gamma - 1) == pytest.approx(u + 2 * cs / (gamma - 1), rel=1e-10)
    # inside the fan the same invariant and entropy hold
    s = np.linspace(uL - cL, u - cs, 7)[1:-1]
    ro, uo, po = riemann.sample(left, right, gamma, s)
    co = np.sqrt(gamma * po / ro)
    assert np.allclose(uo + 2 * co / (gamma - 1), uL + 2 * cL / (gamma - 1), rtol=1e-12)
    assert np.allclose(po / ro ** gamma, pL / rL ** gamma, rtol=1e-12)
    assert np.allclose(uo - co, s, rtol=1e-12, atol=1e-12)  # C- characteristics


def test_far_field_and_contact():
    left, right, gamma = (4, 0, 4), (1, 0, 1), 1.4
    p, u, rl, rr = riemann.star_state(left, right, gamma)
    ro, uo, po = riemann.sample(left, right, gamma, np.array([-10.0, u - 1e-9, u + 1e-9, 10.0]))
    assert (ro[0], uo[0], po[0]) == (4, 0, 4) and (ro[-1], uo[-1], po[-1]) == (1, 0, 1)
    assert po[1] == po[2] == p and uo[1] == uo[2] == u
    assert ro[1] == rl and ro[2] == rr


def test_l1_rel_error_definition():
    from oracle.metrics import l1_rel_error
    assert l1_rel_error([1.0, 2.0, 4.0], [1.0, 2.5, 3.0]) == pytest.approx(1.5 / 6.5)
