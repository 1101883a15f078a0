"""Pins of the oracle's finite-difference update (Sec. V A written for the
translational populations as well; reading B of the translational update).

The pins come from the mathematics of the stencil, not from the code: for a
Fourier mode e^{i theta x} the third-order upwind difference is the mode
times a symbol S(theta) fixed by the stencil coefficients, so one forward
Euler step multiplies each population's mode by G = 1 - nu S(theta) (in 2-D
by 1 - nu_x S(theta_x) - nu_y S(theta_y)) when collisions are switched off.
A dropped term, a wrong coefficient, a wrong upwind orientation or a wrong
Courant number (lambda c_i) changes G."""
import numpy as np
import pytest


def _symbol(theta, nu):
    """Fourier symbol of the third-order upwind difference of Sec. V A."""
    e = np.exp(1j * theta)
    if nu >= 0:  # (h[-2] - 6 h[-1] + 3 h[0] + 2 h[1]) / 6
        return (e ** -2 - 6 * e ** -1 + 3 + 2 * e) / 6
    return (-e ** 2 + 6 * e - 3 - 2 / e) / 6  # (-h[2] + 6 h[1] - 3 h[0] - 2 h[-1]) / 6


@pytest.mark.parametrize("lam", [0.1, 1.0 / 6.0, 1.0])
def test_fd_single_mode_amplification_1d(orc, lam):
    N, k, steps = 64, 3, 5
    theta = 2 * np.pi * k / N
    x = np.arange(N)
    G = orc.Grid(orc.D1Q7, (N,), bc=[orc.PERIODIC], n_rot=2.0, tau=1e300, fd_courant=lam)
    f, g = G.init_eq(np.ones(N), np.zeros((1, N)), np.ones(N))
    c, _, _ = orc.lattice(orc.D1Q7)
    rng = np.random.default_rng(0)
    amp = rng.normal(size=7) + 1j * rng.normal(size=7)
    f0 = f.copy()
    f += np.real(amp[:, None] * np.exp(1j * theta * x)[None, :])
    G.step(f, g, steps)
    for i in range(7):
        nu = lam * c[i, 0]
        grown = amp[i] * (1 - nu * _symbol(theta, nu)) ** steps
        want = f0[i] + np.real(grown * np.exp(1j * theta * x))
        assert np.abs(f[i] - want).max() < 1e-12 * max(1.0, abs(grown)), i


def test_fd_single_mode_amplification_2d(orc):
    nx, ny, lam, steps = 40, 24, 0.12, 4
    tx, ty = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))  # node index x + nx*y
    mode = np.exp(1j * (tx * X + ty * Y)).reshape(-1)
    for kind in (orc.D2Q49, orc.D2Q37):
        G = orc.Grid(kind, (nx, ny), bc=[orc.PERIODIC, orc.PERIODIC], n_rot=3.0, tau=1e300, fd_courant=lam)
        N = nx * ny
        f, g = G.init_eq(np.ones(N), np.zeros((2, N)), np.ones(N))
        c, _, _ = orc.lattice(kind)
        Q = len(c)
        amp = np.random.default_rng(1).normal(size=Q) * (1 + 0.5j)
        f0 = f.copy()
        f += np.real(amp[:, None] * mode[None, :])
        G.step(f, g, steps)
        for i in range(Q):
            nux, nuy = lam * c[i, 0], lam * c[i, 1]
            amp_g = 1 - nux * _symbol(tx, nux) - nuy * _symbol(ty, nuy)
            want = f0[i] + np.real(amp[i] * amp_g ** steps * mode)
            assert np.abs(f[i] - want).max() < 1e-12, (kind, i)


def test_fd_amplification_growth():
    """Forward Euler with the third-order upwind difference amplifies some
    mode at every Courant number (weakly: growth ~nu^3 per step), strongly at
    the streaming time step: at lambda = 1 the fastest populations (|c| = 3,
    nu = 3) grow by more than 4x per step, so the finite-difference reading
    cannot run at the time step the paper's results use; at nu = 0.3 (lambda
    = 0.1) the growth is ~2 % per step, which the collisions must absorb."""
    theta = np.linspace(0.01, np.pi, 400)

    def gmax(nu):
        return np.abs(1 - nu * np.array([_symbol(t, nu) for t in theta])).max()

    assert gmax(3.0) > 4.0 and gmax(-3.0) > 4.0
    assert 1.0 < gmax(0.3) < 1.03 and 1.0 < gmax(0.5) < 1.1
    assert gmax(0.05) - 1.0 < (gmax(0.5) - 1.0) / 300  # ~nu^3


def test_fd_conserves_mass_and_keeps_uniform_states(orc):
    N = 50
    G = orc.Grid(orc.D1Q7, (N,), bc=[orc.PERIODIC], n_rot=4.0, tau=0.7, fd_courant=0.15)
    x = np.arange(N) / N
    f, g = G.init_eq(1 + 0.1 * np.sin(2 * np.pi * x), 0.1 * np.cos(2 * np.pi * x)[None, :],
                     1 + 0.05 * np.sin(4 * np.pi * x))
    m0 = G.moments(f, g)[3]
    G.step(f, g, 40)
    tot = G.moments(f, g)[3]
    assert abs(tot[0] - m0[0]) <= 1e-12 * m0[0]
    # a uniform moving state is a fixed point (zero differences, equilibrium)
    G2 = orc.Grid(orc.D1Q7, (N,), bc=[orc.OPEN], n_rot=4.0, tau=0.7, fd_courant=0.15)
    f2, g2 = G2.init_eq(np.full(N, 1.3), np.full((1, N), 0.2), np.full(N, 0.9))
    ff, gg = f2.copy(), g2.copy()
    G2.step(f2, g2, 10)
    assert np.abs(f2 - ff).max() < 1e-13 and np.abs(g2 - gg).max() < 1e-13
