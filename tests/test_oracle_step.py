"""Pins of the oracle's moments, collision, streaming and rotational
advection (Sec. V) against invariants, brute force and closed forms."""
import numpy as np
import pytest

BIG_TAU = 1e300  # omega = 1e-300: the BGK term is below one ulp, so f* == f


def _rand_state(orc, G, seed, amp=0.05):
    """Equilibrium of a smooth random field plus a small random
    non-equilibrium part, so collisions have something to relax."""
    rng = np.random.default_rng(seed)
    N, D = G.N, G.D
    rho = 1.0 + amp * rng.uniform(-1, 1, N)
    u = 0.1 * rng.uniform(-1, 1, (D, N))
    T = 1.0 + amp * rng.uniform(-1, 1, N)
    f, g = G.init_eq(rho, u, T)
    f *= 1.0 + 0.01 * rng.uniform(-1, 1, f.shape)
    g *= 1.0 + 0.01 * rng.uniform(-1, 1, g.shape)
    return f, g


@pytest.mark.parametrize("kind,shape", [("D1Q7", (1,)), ("D2Q49", (1, 1)),
                                        ("D2Q37", (1, 1)), ("D3Q343", (1, 1, 1))])
@pytest.mark.parametrize("n_rot", [0.0, 3.0, 11.0 / 3.0])
def test_temperature_round_trip(orc, kind, shape, n_rot):
    G = orc.Grid(getattr(orc, kind), shape, n_rot=n_rot, tau=1.0)
    for rho, u, T in [(1.3, 0.2, 0.9), (0.6, -0.35, 1.4)]:
        uu = np.full((G.D, 1), u)
        f, g = G.init_eq(np.array([rho]), uu, np.array([T]))
        r_, u_, T_, tot = G.moments(f, g)
        assert r_[0] == pytest.approx(rho, rel=1e-14)
        assert np.allclose(u_[:, 0], u, rtol=1e-13)
        assert T_[0] == pytest.approx(T, rel=1e-13)
        # total energy = rho (|u|^2/2 + (D+n) T / 2)   (Sec. II, internal energy E)
        assert tot[-1] == pytest.approx(rho * (0.5 * G.D * u * u + 0.5 * (G.D + n_rot) * T),
                                        rel=1e-13)


@pytest.mark.parametrize("kind,shape", [("D1Q7", (1,)), ("D2Q49", (1, 1)),
                                        ("D2Q37", (1, 1)), ("D3Q343", (1, 1, 1))])
@pytest.mark.parametrize("n_rot", [0.0, 2.0, 4.0])
def test_collision_conserves_mass_momentum_energy(orc, kind, shape, n_rot):
    # A one-node periodic grid streams every population onto itself and the
    # upwind differences vanish, so a step is the bare collision.
    G = orc.Grid(getattr(orc, kind), shape, n_rot=n_rot, tau=0.8)
    f, g = _rand_state(orc, G, 7)
    before = G.moments(f, g)[3]
    G.step(f, g, 1)
    after = G.moments(f, g)[3]
    assert np.allclose(after, before, rtol=1e-14, atol=1e-15)


def test_collision_relaxes_towards_equilibrium(orc):
    G = orc.Grid(orc.D1Q7, (1,), n_rot=2.0, tau=2.0)
    f, g = _rand_state(orc, G, 3)
    rho, u, T, _ = G.moments(f, g)
    fe = orc.feq(orc.D1Q7, rho[0], u[:, 0], T[0])
    ge = orc.geq(T[0])
    f1, g1 = f.copy(), g.copy()
    G.step(f1, g1, 1)
    # f* = f - (f - f^eq)/tau ; g' = g - (g - g^eq)/tau  (one node, no advection)
    assert np.allclose(f1[:, 0], f[:, 0] - 0.5 * (f[:, 0] - fe), rtol=1e-14, atol=1e-16)
    assert np.allclose(g1[:, 0], g[:, 0] - 0.5 * (g[:, 0] - ge), rtol=1e-14, atol=1e-16)


def _stream_case(orc, kind, shape, bc):
    G = orc.Grid(getattr(orc, kind), shape, bc=bc, n_rot=0.0, tau=BIG_TAU)
    N = G.N
    f, g = G.init_eq(np.ones(N), np.zeros((G.D, N)), np.ones(N))
    rng = np.random.default_rng(11)
    f += 1e-3 * rng.uniform(0, 1, f.shape)  # distinct labels on every population
    return G, f, g


@pytest.mark.parametrize("bc", [0, 1])
def test_streaming_brute_force_1d(orc, bc):
    G, f, g = _stream_case(orc, "D1Q7", (5,), (bc,))
    c, _, _ = orc.lattice(orc.D1Q7)
    f0 = f.copy()
    G.step(f, g, 1)
    for i in range(7):
        for x in range(5):
            src = x - c[i, 0]
            src = src % 5 if bc == 0 else min(max(src, 0), 4)
            assert f[i, x] == f0[i, src]


@pytest.mark.parametrize("bc", [(0, 0), (1, 0), (0, 1)])
def test_streaming_brute_force_2d(orc, bc):
    nx, ny = 4, 5
    G, f, g = _stream_case(orc, "D2Q49", (nx, ny), bc)
    c, _, _ = orc.lattice(orc.D2Q49)
    f0 = f.copy()
    G.step(f, g, 1)

    def S(v, n, b):
        return v % n if b == 0 else min(max(v, 0), n - 1)
    for i in range(49):
        for y in range(ny):
            for x in range(nx):
                sx, sy = S(x - c[i, 0], nx, bc[0]), S(y - c[i, 1], ny, bc[1])
                assert f[i, x + nx * y] == f0[i, sx + nx * sy]


def test_streaming_brute_force_3d(orc):
    G, f, g = _stream_case(orc, "D3Q343", (3, 4, 2), (0, 1, 0))
    c, _, _ = orc.lattice(orc.D3Q343)
    f0 = f.copy().reshape(343, 2, 4, 3)
    G.step(f, g, 1)
    f = f.reshape(343, 2, 4, 3)
    for i in range(343):
        for z in range(2):
            for y in range(4):
                for x in range(3):
                    sx = (x - c[i, 0]) % 3
                    sy = min(max(y - c[i, 1], 0), 3)
                    sz = (z - c[i, 2]) % 2
                    assert f[i, z, y, x] == f0[i, sz, sy, sx]


@pytest.mark.parametrize("u0", [0.3, -0.45])
def test_upwind_exact_for_cubics(orc, u0):
    # Uniform flow u0 with no relaxation: g' = g - nu * d/dx g exactly for
    # cubic g at nodes at least two away from the open ends (Sec. V A).
    N = 24
    G = orc.Grid(orc.D1Q7, (N,), bc=(1,), n_rot=0.0, tau=BIG_TAU)
    f, g = G.init_eq(np.ones(N), np.full((1, N), u0), np.ones(N))
    x = np.arange(N, dtype=np.float64)
    poly = 0.3 + 0.02 * x - 0.004 * x ** 2 + 0.0005 * x ** 3
    dpoly = 0.02 - 0.008 * x + 0.0015 * x ** 2
    for j in range(7):
        g[j] = poly * (j + 1)
    G.step(f, g, 1)
    nu = u0 / orc.d1q7_r()
    for j in range(7):
        want = (poly - nu * dpoly) * (j + 1)
        assert np.allclose(g[j, 2:-2], want[2:-2], rtol=0, atol=1e-13)


def test_upwind_third_order_convergence(orc):
    errs = []
    for N in (32, 64, 128):
        G = orc.Grid(orc.D1Q7, (N,), bc=(0,), n_rot=0.0, tau=BIG_TAU)
        f, g = G.init_eq(np.ones(N), np.full((1, N), 0.4), np.ones(N))
        x = np.arange(N) / N
        h = np.sin(2 * np.pi * x)
        g[:] = h
        G.step(f, g, 1)
        exact_d = 2 * np.pi / N * np.cos(2 * np.pi * x)  # d/d(node index)
        nu = 0.4 / orc.d1q7_r()
        errs.append(np.abs(g[0] - (h - nu * exact_d)).max())
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    # one step's error is nu * (spatial error) = O(dx^4) per unit step in
    # node units -> ratio 2^4 per halving of the node spacing
    assert np.all(np.abs(slopes - 4.0) < 0.2), slopes


@pytest.mark.parametrize("kind,shape,bc", [("D1Q7", (16,), (0,)), ("D1Q7", (16,), (1,)),
                                           ("D2Q49", (6, 5), (0, 1)), ("D2Q37", (6, 5), (1, 0)),
                                           ("D3Q343", (4, 3, 3), (0, 0, 1))])
def test_uniform_state_is_invariant(orc, kind, shape, bc):
    G = orc.Grid(getattr(orc, kind), shape, bc=bc, n_rot=3.0, tau=0.7)
    N = G.N
    u = np.zeros((G.D, N))
    u[0] = 0.2
    if G.D > 1:
        u[1] = -0.1
    f, g = G.init_eq(np.full(N, 1.2), u, np.full(N, 0.95))
    f0, g0 = f.copy(), g.copy()
    G.step(f, g, 20)
    # rounding of the moment round trip only: well below 1e-14 of the largest
    # population per step
    assert np.abs(f - f0).max() <= 20 * 1e-14 * f0.max()
    assert np.abs(g - g0).max() <= 20 * 1e-14 * g0.max()


@pytest.mark.parametrize("n_rot", [0.0, 3.0])
def test_periodic_conservation_2d(orc, n_rot):
    G = orc.Grid(orc.D2Q49, (12, 10), n_rot=n_rot, tau=0.9)
    f, g = _rand_state(orc, G, 5)
    t0 = G.moments(f, g)[3]
    G.step(f, g, 50)
    t1 = G.moments(f, g)[3]
    assert t1[0] == pytest.approx(t0[0], rel=1e-13)
    assert np.allclose(t1[1:3], t0[1:3], rtol=0, atol=1e-12 * t0[0])
    if n_rot == 0.0:
        # the rotational populations carry no energy when n = 0, and the
        # collision and the streaming conserve the rest exactly
        assert t1[3] == pytest.approx(t0[3], rel=1e-13)
    else:
        # the upwind advection of g is not in conservation form, so energy
        # changes at truncation level (node-to-node random fields here)
        assert t1[3] != t0[3]
        assert t1[3] == pytest.approx(t0[3], rel=1e-3)


def test_energy_drift_shrinks_with_resolution(orc):
    # n > 0: the non-conservative rotational advection changes the total
    # energy at truncation level; for a smooth field the drift falls with
    # resolution (about first order: the viscosity in node units is fixed).
    drifts = []
    for N in (32, 128):
        G = orc.Grid(orc.D1Q7, (N,), n_rot=3.0, tau=0.8)
        x = np.arange(N) / N
        f, g = G.init_eq(1 + 0.05 * np.sin(2 * np.pi * x),
                         (0.1 * np.cos(2 * np.pi * x))[None], 1 + 0.05 * np.cos(2 * np.pi * x))
        e0 = G.moments(f, g)[3][-1]
        G.step(f, g, N)  # same physical time
        drifts.append(abs(G.moments(f, g)[3][-1] - e0) / e0)
    assert drifts[1] < 0.5 * drifts[0]
