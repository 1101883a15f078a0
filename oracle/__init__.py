"""FP64 CPU oracle of the decoupled Hermite lattice Boltzmann scheme.

TEST INFRASTRUCTURE ONLY: the reference the GPU path is checked against.
Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code, header, table or
constant with the GPU library (`paper_1606_06107_amd`), and never imports it.

Contents
  lbm_oracle.c   plain C scalar loops (lattices, equilibria, moments, one
                 time step, boundary conditions, totals), loaded via ctypes
  riemann.py     exact Riemann solver for an ideal gas (Sod reference)
  metrics.py     the relative L1 error of Sec. VI
  surrogate_ref.py  FP64 NumPy forward/backward of the learned surrogate

Naming: ``f`` = translational populations (the paper's g_i), ``g`` =
rotational populations (the paper's h_j).  Arrays are [Q][N] with the node
index x fastest (x + nx*(y + ny*z)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# LBMX_ORACLE_LIB names another build of the same source (the sanitizer
# build of the test suite's address/undefined-behaviour check).
_LIB_LOAD = os.environ.get("LBMX_ORACLE_LIB") or _LIB

D1Q7, D2Q49, D3Q343, D2Q37 = 1, 2, 3, 4
PERIODIC, OPEN = 0, 1
_QOF = {D1Q7: 7, D2Q49: 49, D3Q343: 343, D2Q37: 37}
_DIMOF = {D1Q7: 1, D2Q49: 2, D3Q343: 3, D2Q37: 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3, OpenMP).  Compiling it does not load
    it; the library is only loaded by `lib()`.

    ISO C mode (-std=c99) keeps multiply-adds unfused (-ffp-contract=off), so
    the arithmetic is the one written, whatever the instruction set.  The
    instruction set is x86-64-v4 (AVX-512) rather than the build host's own
    (-march=native): the library is compiled on one machine and runs on
    another host CPU as well."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v4", "-std=c99", "-ffp-contract=off",
                               "-fPIC", "-shared", "-fopenmp", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("lattice", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("bc", ctypes.c_int32 * 3),
                ("n_rot", ctypes.c_double), ("tau", ctypes.c_double),
                ("fd_courant", ctypes.c_double), ("g_substeps", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_LOAD == _LIB and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB_LOAD)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_d1q7_r.restype = ctypes.c_double
        L.orc_lattice.argtypes = [ctypes.c_int, ip, dp, dp]
        L.orc_feq.argtypes = [ctypes.c_int, ctypes.c_int, ip, dp, ctypes.c_double,
                              ctypes.c_double, dp, ctypes.c_double, dp]
        L.orc_geq.argtypes = [ctypes.c_double, dp]
        gp = ctypes.POINTER(_Grid)
        L.orc_init_eq.argtypes = [gp, dp, dp, dp, dp, dp]
        L.orc_step.argtypes = [gp, dp, dp, dp, dp, ctypes.c_int64]
        L.orc_moments.argtypes = [gp, dp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def d1q7_r() -> float:
    """Scaling factor r of the D1Q7 Gauss-Hermite model (Table II)."""
    return lib().orc_d1q7_r()


def lattice(kind: int):
    """(c[Q,3] int, w[Q], r) of a translational lattice (Tables I, II)."""
    Q = _QOF[kind]
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    r = ctypes.c_double()
    q = lib().orc_lattice(kind, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w),
                          ctypes.byref(r))
    assert q == Q
    return c, w, r.value


def rot_lattice():
    """(eta[7], w[7]) of the rotational D1Q7 model (Table II)."""
    c, w, r = lattice(D1Q7)
    return r * c[:, 0].astype(np.float64), w


def feq(kind: int, rho: float, u, theta: float) -> np.ndarray:
    """Translational equilibrium populations of one node (Sec. IV)."""
    c, w, r = lattice(kind)
    D = _DIMOF[kind]
    uu = np.zeros(3)
    uu[:len(u)] = u
    out = np.zeros(len(w))
    lib().orc_feq(D, len(w), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w), r,
                  float(rho), _dp(uu), float(theta), _dp(out))
    return out


def geq(theta: float) -> np.ndarray:
    """Rotational equilibrium populations (Sec. IV)."""
    out = np.zeros(7)
    lib().orc_geq(float(theta), _dp(out))
    return out


class Grid:
    """A grid of nodes with one lattice, boundary conditions, n and tau.
    fd_courant = 0: the collide-and-stream update; lambda > 0: the
    finite-difference update of Sec. V A for f as well, with time step
    lambda times the streaming step (tau stays in streaming steps).
    g_substeps = m > 1 splits the rotational advection into m sub-steps of
    Courant number u_a / (m r) (not the paper's update: a diagnostic that
    separates its Courant limit from other causes of divergence)."""

    def __init__(self, lattice_kind: int, shape, bc=(PERIODIC, PERIODIC, PERIODIC),
                 n_rot: float = 0.0, tau: float = 1.0, fd_courant: float = 0.0, g_substeps: int = 1):
        D = _DIMOF[lattice_kind]
        shape = tuple(int(s) for s in shape)
        assert len(shape) == D, "shape must have one entry per spatial dimension"
        n = list(shape) + [1] * (3 - D)
        bcs = list(bc)[:D] + [PERIODIC] * (3 - D)
        self.kind, self.D, self.Q = lattice_kind, D, _QOF[lattice_kind]
        self.shape, self.N = shape, int(np.prod(shape))
        self.n_rot, self.tau = float(n_rot), float(tau)
        self.fd_courant = float(fd_courant)
        self._g = _Grid(D, lattice_kind, (ctypes.c_int64 * 3)(*n), (ctypes.c_int32 * 3)(*bcs),
                        self.n_rot, self.tau, self.fd_courant, int(g_substeps))

    def init_eq(self, rho, u, T):
        """f = f^eq(rho, u, T), g = g^eq(T) at every node.  u is [D][N]."""
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.N)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.D, self.N)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.N)
        f = np.zeros((self.Q, self.N))
        g = np.zeros((7, self.N))
        rc = lib().orc_init_eq(ctypes.byref(self._g), _dp(rho), _dp(u), _dp(T), _dp(f), _dp(g))
        assert rc == 0
        return f, g

    def step(self, f, g, nsteps: int = 1):
        """Advance (f, g) in place by nsteps time steps."""
        assert f.shape == (self.Q, self.N) and g.shape == (7, self.N)
        fs = np.empty_like(f)
        gs = np.empty_like(g)
        rc = lib().orc_step(ctypes.byref(self._g), _dp(f), _dp(g), _dp(fs), _dp(gs),
                            int(nsteps))
        if rc != 0:
            raise ValueError(f"orc_step failed ({rc})")
        return f, g

    def moments(self, f, g):
        """(rho[N], u[D,N], T[N], totals[2+D]) with totals = mass, momentum, energy."""
        rho = np.zeros(self.N)
        u = np.zeros((self.D, self.N))
        T = np.zeros(self.N)
        tot = np.zeros(2 + self.D)
        rc = lib().orc_moments(ctypes.byref(self._g), _dp(f), _dp(g), _dp(rho), _dp(u),
                               _dp(T), _dp(tot))
        assert rc == 0
        return rho, u, T, tot


def set_threads(n: int) -> int:
    """Thread count of the OpenMP node loops (results do not depend on it).
    Returns the count now in use."""
    return int(lib().orc_set_threads(int(n)))
