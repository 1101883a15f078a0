"""Pins of the whole oracle time step against closed-form flow physics:
shear-wave decay, the acoustic speed that fixes gamma = (D+n+2)/(D+n)
(Sec. III), the shock-tube analytical solution (Sec. VI) and the paper's own
worked example (Sec. VI, Table III)."""
import math

import numpy as np
import pytest

from conftest import golden


def test_shear_wave_viscosity(orc):
    # Exact streaming with BGK: nu = c_s^2 (tau - 1/2) in node units with
    # c_s^2 = T / r^2 (xi = r c).  u_y = A sin(k x) decays as exp(-nu k^2 t).
    L, tau, T0, A = 64, 0.8, 1.0, 0.01
    G = orc.Grid(orc.D2Q49, (L, 1), n_rot=3.0, tau=tau)
    x = np.arange(L)
    u = np.zeros((2, L))
    u[1] = A * np.sin(2 * np.pi * x / L)
    f, g = G.init_eq(np.ones(L), u, np.full(L, T0))
    amps = []
    for t_target in (50, 300):
        G.step(f, g, t_target - (50 if amps else 0))
        uy = G.moments(f, g)[1][1]
        amps.append(abs(np.fft.rfft(uy)[1]))
    rate = math.log(amps[0] / amps[1]) / 250.0
    r = orc.d1q7_r()
    k = 2 * np.pi / L
    nu = T0 / r ** 2 * (tau - 0.5)
    assert rate == pytest.approx(nu * k * k, rel=0.01)


@pytest.mark.parametrize("n_rot", [0.0, 2.0, 4.0, 11.0 / 3.0, 19.0])
def test_acoustic_speed_gives_gamma(orc, n_rot):
    # A right-moving linear sound wave travels at c = sqrt(gamma T0) in the
    # paper's units, i.e. c / r nodes per step.
    L, T0, A, tau = 128, 1.0, 1e-4, 0.6
    D = 1
    gamma = (D + n_rot + 2) / (D + n_rot)
    r = orc.d1q7_r()
    c = math.sqrt(gamma * T0)
    x = np.arange(L)
    s = A * np.cos(2 * np.pi * x / L)
    G = orc.Grid(orc.D1Q7, (L,), n_rot=n_rot, tau=tau)
    f, g = G.init_eq(1 + s, (c * s)[None], T0 * (1 + (gamma - 1) * s))
    phases, times = [], []
    for t in range(0, 201, 20):
        if t:
            G.step(f, g, 20)
        rho = G.moments(f, g)[0]
        phases.append(np.angle(np.fft.fft(rho)[1]))
        times.append(t)
    ph = np.unwrap(phases)
    slope = np.polyfit(times, ph, 1)[0]
    v = -slope / (2 * np.pi / L)  # nodes per step
    gamma_meas = (v * r) ** 2 / T0
    assert gamma_meas == pytest.approx(gamma, rel=0.005)


def _tube(orc, N, left, right, n_rot, tau, steps, kind=None, ny=None):
    from oracle import riemann
    from oracle.metrics import l1_rel_error
    r = orc.d1q7_r()
    x = (np.arange(N) + 0.5) / N  # cell-centred, diaphragm at x = 1/2
    rho = np.where(x < 0.5, left[0], right[0])
    T = np.where(x < 0.5, left[2] / left[0], right[2] / right[0])
    if ny:
        G = orc.Grid(kind, (N, ny), bc=(orc.OPEN, orc.PERIODIC), n_rot=n_rot, tau=tau)
        f, g = G.init_eq(np.tile(rho, ny), np.zeros((2, N * ny)), np.tile(T, ny))
    else:
        G = orc.Grid(orc.D1Q7, (N,), bc=(orc.OPEN,), n_rot=n_rot, tau=tau)
        f, g = G.init_eq(rho, np.zeros((1, N)), T)
    G.step(f, g, steps)
    rr, uu, TT, _ = G.moments(f, g)
    if ny:
        row = ny // 2
        rr, TT, ux = (a.reshape(ny, N)[row] for a in (rr, TT, uu[0]))
        for a in (G.moments(f, g)[0].reshape(ny, N),):
            assert np.allclose(a, a[row], rtol=1e-12)  # uniform across the periodic axis
    else:
        ux = uu[0]
    Dm = 2 if ny else 1
    gamma = (Dm + n_rot + 2) / (Dm + n_rot)
    t = steps / (N * r)  # Sec. VI: t = step / (X r)
    ra, ua, pa = riemann.sample(left, right, gamma, (x - 0.5) / t)
    return {"rho": l1_rel_error(rr, ra), "p": l1_rel_error(rr * TT, pa),
            "T": l1_rel_error(TT, pa / ra), "u_x": l1_rel_error(ux, ua)}


@pytest.mark.parametrize("steps", [180, 239])
def test_shock_tube_1d_vs_exact_riemann(orc, steps):
    # The paper's tube (rho 4:1, T = 1) in 1-D with n = 4 (gamma = 1.4).
    e = _tube(orc, 1000, (4.0, 0.0, 4.0), (1.0, 0.0, 1.0), 4.0, 2.0 / 3.0, steps)
    assert e["rho"] < 2e-2 and e["p"] < 2e-2 and e["T"] < 2e-2 and e["u_x"] < 4e-2, e


@pytest.mark.slow
def test_paper_worked_example_table3(orc):
    # Sec. VI exactly: D2Q37 + D1Q7 on 1000 x 16, open in x, periodic in y,
    # n = 3, tau = 2/3, step 180.  The paper's errors (Table III) come from a
    # code we do not have; agreement within a factor 2 either way confirms
    # the collide-and-stream reading of the translational update.
    e = _tube(orc, 1000, (4.0, 0.0, 4.0), (1.0, 0.0, 1.0), 3.0, 2.0 / 3.0, 180,
              kind=orc.D2Q37, ny=16)
    table = {k: float(v) for k, v in golden("table3_errors.txt")}
    for k, v in table.items():
        assert v / 2.0 <= e[k] <= 2.0 * v, (k, e[k], v)


@pytest.mark.parametrize("n_rot", [0.0, 2.0, 6.0])
def test_heat_diffusivity_translational_only(orc, n_rot):
    # An isobaric temperature wave (rho T = const, u = 0) decays as
    # exp(-chi k^2 t).  Only the translational populations move relative to
    # the fluid (the rotational ones are advected with u), so the heat flux
    # is that of the D+2 translational degrees of freedom while the heat
    # capacity counts all D+n+2: chi = (D+2)/(D+n+2) (T/r^2)(tau - 1/2),
    # i.e. (D+2)/(D+n+2) of the conductivity of the paper's Chapman-Enskog
    # result (Sec. II), whose Prandtl number is 1.
    L, tau, T0, eps, D = 64, 0.8, 1.0, 0.01, 2
    G = orc.Grid(orc.D2Q49, (L, 3), n_rot=n_rot, tau=tau)
    x = np.tile(np.arange(L), 3)
    k = 2 * np.pi / L
    s = np.sin(k * x)
    f, g = G.init_eq(1 / (1 + eps * s), np.zeros((2, 3 * L)), T0 * (1 + eps * s))
    amps = []
    for _ in range(6):
        G.step(f, g, 100)
        amps.append(2 * abs(np.mean(G.moments(f, g)[2] * np.exp(-1j * k * x))))
    t = 100 * np.arange(1, 7)
    chi = -np.polyfit(t[2:], np.log(amps[2:]), 1)[0] / k ** 2
    nu = T0 / orc.d1q7_r() ** 2 * (tau - 0.5)
    assert chi == pytest.approx((D + 2) / (D + n_rot + 2) * nu, rel=4e-2)
    if n_rot > 0:
        assert abs(chi / nu - 1.0) > 0.3  # not the paper's Pr = 1


@pytest.mark.parametrize("pl,pr,dl,dr,n_rot", [(1.0, 0.1, 1.0, 0.125, 4.0), (1.0, 0.5, 1.0, 0.5, 2.0),
                                               (1.0, 1.0, 1.0, 0.5, 4.0)])
def test_open_tube_momentum_balance(orc, pl, pr, dl, dr, n_rot):
    # Integrated over an open tube, the momentum equation (Sec. II) says the
    # total momentum changes only by the pressure at the two ends.  With
    # exact streaming a population moves c = xi / r nodes per step and
    # carries xi, so the momentum crossing a cut per step is
    # sum f xi^2 / r = rho (u^2 + T) / r: at rest ends, K steps add
    # (K / r)(p_l - p_r) while mass stays.  Pins the clamped open boundary
    # of both population sets (a wrong clamp leaks mass or momentum).
    L, K = 400, 16
    G = orc.Grid(orc.D1Q7, (L,), bc=(orc.OPEN,), n_rot=n_rot, tau=0.8)
    left = np.arange(L) < L // 2
    rho = np.where(left, dl, dr)
    T = np.where(left, pl / dl, pr / dr)
    f, g = G.init_eq(rho, np.zeros((1, L)), T)
    r0, u0, _, _ = G.moments(f, g)
    G.step(f, g, K)
    r1, u1, T1, _ = G.moments(f, g)
    # the waves stay far from the ends over K steps
    assert abs(u1[0][0]) < 1e-12 and abs(u1[0][-1]) < 1e-12
    assert r1.sum() == pytest.approx(r0.sum(), rel=1e-13)
    dP = (r1 * u1[0]).sum() - (r0 * u0[0]).sum()
    assert dP == pytest.approx(K / orc.d1q7_r() * (pl - pr), rel=1e-10, abs=1e-12)


def test_classic_sod_diverges_through_the_rotational_courant_limit(orc):
    """The classic Sod tube (1,0,1) | (0.125,0,0.1), n = 4, tau = 1: its
    star state moves at u* = 0.93 (rotational Courant number 0.78, above the
    0.67 where the rotational update of Sec. V A stays linearly stable at
    tau = 1).  With that update as written the tube diverges within 100
    steps; with the same advection in 4 sub-steps (Courant 0.19) it stays
    finite and positive over 1000 steps and matches the exact Riemann
    solution at t = 0.2 at the level of Table III.  So the divergence is the
    rotational update's Courant limit, not a loss of positivity of the
    translational equilibrium."""
    import workloads
    from oracle import riemann
    from oracle.metrics import l1_rel_error as rel_l1
    N = 1000
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    rho, u, T = workloads.sod_tube(N, left, right)

    def run(m, steps):
        G = orc.Grid(orc.D1Q7, (N,), bc=(orc.OPEN,), n_rot=4.0, tau=1.0, g_substeps=m)
        f, g = G.init_eq(rho, u, T)
        for k in range(0, steps, 10):
            G.step(f, g, 10)
            r, uu, TT, _ = G.moments(f, g)
            if not (np.isfinite(TT).all() and r.min() > 0 and TT.min() > 0):
                return k + 10, None
        return None, (r, uu, TT)

    died, _ = run(1, 100)
    assert died is not None and died <= 100
    died, (r, uu, TT) = run(4, 240)
    assert died is None
    # 240 steps run in chunks of 10: the state at step 240; compare at that time
    x = (np.arange(N) + 0.5) / N
    t = 240 / (N * orc.d1q7_r())
    ra, ua, pa = riemann.sample(left, right, 1.4, (x - 0.5) / t)
    assert rel_l1(r, ra) < 0.015 and rel_l1(uu[0], ua) < 0.035 and rel_l1(r * TT, pa) < 0.015
    died, _ = run(4, 1000)
    assert died is None


@pytest.mark.parametrize("m", [2, 5])
def test_substeps_keep_invariants(orc, m):
    """The sub-stepped rotational advection keeps what the update keeps: a
    uniform state is invariant, and a periodic grid conserves mass and
    momentum to rounding (they are moments of the translational populations
    only); with n = 0 energy as well."""
    shape = (24, 18)
    N = 24 * 18
    G = orc.Grid(orc.D2Q49, shape, n_rot=2.0, tau=0.8, g_substeps=m)
    uu = np.zeros((2, N))
    uu[0], uu[1] = 0.3, -0.2
    f, g = G.init_eq(np.full(N, 1.1), uu, np.full(N, 0.9))
    G.step(f, g, 20)
    r, u2, T, _ = G.moments(f, g)
    assert np.abs(r - 1.1).max() < 1e-13 and np.abs(T - 0.9).max() < 1e-12 and np.abs(u2[0] - 0.3).max() < 1e-13
    rng = np.random.default_rng(3)
    rho = 1 + 0.05 * rng.standard_normal(N)
    uu = 0.05 * rng.standard_normal((2, N))
    T = 1 + 0.05 * rng.standard_normal(N)
    for n_rot in (2.0, 0.0):
        G = orc.Grid(orc.D2Q49, shape, n_rot=n_rot, tau=0.8, g_substeps=m)
        f, g = G.init_eq(rho, uu, T)
        t0 = G.moments(f, g)[3]
        G.step(f, g, 30)
        t1 = G.moments(f, g)[3]
        assert np.abs(t1[:3] - t0[:3]).max() < 1e-12 * t0[0]
        if n_rot == 0.0:
            assert abs(t1[3] - t0[3]) < 1e-12 * t0[3]
