"""Seeded synthetic inputs shared by the tests, the benchmark and the
surrogate's data generation.

This module holds no arithmetic of the lattice Boltzmann method: it only
draws macroscopic initial fields (rho, u, T) and per-instance parameters with
NumPy's ``default_rng(seed)`` in FP64.  Both the CPU oracle and the GPU
library consume what it returns; neither is imported here.

Shapes follow the paper's shock-tube test (Sec. VI) and the workloads the
library is measured on:

  sod_tube          1-D tube, cell-centred, diaphragm at x = 1/2
  tube_1d           the classic Sod tube: 1000 nodes, left (rho,u,p) =
                    (1,0,1), right (0.125,0,0.1), n = 4 (gamma = 1.4 in
                    1-D), tau = 1, open ends, 1000 steps, rotational
                    advection in 4 sub-steps
  paper_tube_1d     the Sec. VI tube's states (4,0,4) | (1,0,1) in 1-D,
                    tau = 0.8, the rotational update as written (the paper's
                    tau = 2/3 diverges once the shock leaves the open end)
  periodic_2d       1024^2 smooth random Fourier-mode fields, gamma = 1.4
  turbulence_3d     256^3 solenoidal random velocity, E(k) ~ k^4 exp(-2 (k/4)^2)
  batched_tubes     thousands of ragged 1-D tubes with per-instance gamma,
                    pressure and density ratios, tau and step counts

gamma maps to the rotational degrees of freedom through the paper's relation
gamma = (D+n+2)/(D+n), i.e. n = 2/(gamma-1) - D.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Scaling factor of the D1Q7 set as printed in the caption of Table II; used
# here only to turn a physical end time into a whole number of steps.
R_PRINTED = 1.1969797752


def n_of_gamma(gamma, D: int):
    """Rotational degrees of freedom n = 2/(gamma-1) - D; a result within
    rounding of zero (gamma = 5/3 in 3-D) is exactly zero."""
    n = 2.0 / (np.asarray(gamma, dtype=np.float64) - 1.0) - D
    n = np.where(np.abs(n) < 1e-12, 0.0, n)
    return float(n) if n.ndim == 0 else n


def sod_tube(N: int, left, right):
    """Cell-centred tube on [0,1]: x_k = (k+1/2)/N, left state where x < 1/2.
    left/right = (rho, u, p).  Returns (rho[N], u[1,N], T[N]) with T = p/rho."""
    x = (np.arange(N) + 0.5) / N
    L = x < 0.5
    rho = np.where(L, left[0], right[0]).astype(np.float64)
    u = np.where(L, left[1], right[1]).astype(np.float64)[None, :]
    T = np.where(L, left[2] / left[0], right[2] / right[0]).astype(np.float64)
    return rho, u, T


@dataclass
class Tube1D:
    """The 1-D shock tube workload: the classic Sod states (rho, u, p) =
    (1, 0, 1) | (0.125, 0, 0.1), 1000 cell-centred nodes, open ends, n = 4
    (gamma = 1.4 in 1-D), 1000 steps.  The star state moves at u* = 0.93,
    rotational Courant number 0.78, beyond the ~0.67 where the forward-Euler
    upwind update of the rotational populations stays stable at tau = 1: run
    with that advection in g_substeps = 4 sub-steps (Courant 0.19)."""
    N: int = 1000
    left: tuple = (1.0, 0.0, 1.0)
    right: tuple = (0.125, 0.0, 0.1)
    n_rot: float = 4.0
    tau: float = 1.0
    g_substeps: int = 4
    steps: int = 1000
    riemann_steps: tuple = (180, 239)

    def fields(self):
        return sod_tube(self.N, self.left, self.right)


def tube_1d() -> Tube1D:
    return Tube1D()


def paper_tube_1d() -> Tube1D:
    """The Sec. VI tube's states (rho 4:1 at T = 1) in 1-D: stable with the
    rotational update as written (tau = 0.8)."""
    return Tube1D(left=(4.0, 0.0, 4.0), right=(1.0, 0.0, 1.0), tau=0.8, g_substeps=1)


def _mode_sum(rng, shape, nmodes=8, kmax=4):
    """sum_m a_m cos(2 pi k_m.x / L + phi_m), a ~ U(0,1) normalised to sum 1,
    k_m in {-kmax..kmax}^D without 0, phi ~ U(0, 2 pi)."""
    D = len(shape)
    grids = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    a = rng.uniform(0, 1, nmodes)
    a /= a.sum()
    out = np.zeros(shape)
    for m in range(nmodes):
        while True:
            k = rng.integers(-kmax, kmax + 1, D)
            if np.any(k != 0):
                break
        phi = rng.uniform(0, 2 * np.pi)
        out += a[m] * np.cos(2 * np.pi * sum(k[d] * grids[d] for d in range(D)) + phi)
    return out


@dataclass
class Periodic2D:
    nx: int = 1024
    ny: int = 1024
    gamma: float = 1.4
    tau: float = 1.0
    steps: int = 5000
    mach: float = 0.3
    seed: int = 0

    @property
    def n_rot(self):
        return n_of_gamma(self.gamma, 2)

    def fields(self):
        """(rho[N], u[2,N], T[N]), node index x fastest.  rho = 1 + 0.05 S_rho,
        T = 1 + 0.05 S_T, u from its own mode sums scaled so that
        max |u| / sqrt(gamma T) = mach."""
        shape = (self.ny, self.nx)  # row-major: x fastest
        s = self.seed
        rho = 1.0 + 0.05 * _mode_sum(np.random.default_rng(s), shape)
        ux = _mode_sum(np.random.default_rng(s + 1), shape)
        uy = _mode_sum(np.random.default_rng(s + 2), shape)
        T = 1.0 + 0.05 * _mode_sum(np.random.default_rng(s + 3), shape)
        mach = np.sqrt(ux ** 2 + uy ** 2) / np.sqrt(self.gamma * T)
        scale = self.mach / mach.max()
        u = np.stack([ux * scale, uy * scale]).reshape(2, -1)
        return rho.reshape(-1), u, T.reshape(-1)


@dataclass
class Turbulence3D:
    """tau = 1: the relaxation time of the 3-D workload.  The forward-Euler
    upwind update of the rotational populations is linearly unstable where
    the Courant number |u_a|/r exceeds a bound that falls with 1/tau (0.67 at
    tau = 1, about 0.25 at tau = 0.6), and the initial peak speed here is
    ~0.9 (Courant number 0.75).  Measured on the GPU: tau = 0.6 diverges
    within 100 steps at 128^3 for n > 0 and not for n = 0 (whose rotational
    populations carry no energy); tau = 0.8 diverges at 256^3 in FP32 for n > 0
    within 100 steps while FP64 survives 2000 (the unstable mode grows from
    rounding noise); tau = 1 runs 2000 steps at 256^3 for every gamma."""
    n: int = 256
    gamma: float = 1.4
    tau: float = 1.0
    steps: int = 2000
    mach_rms: float = 0.3
    seed: int = 0

    @property
    def n_rot(self):
        return n_of_gamma(self.gamma, 3)

    def fields(self):
        """Uniform rho = T = 1 and a solenoidal velocity with spectrum
        E(k) ~ k^4 exp(-2 (k/4)^2), scaled to sqrt(<|u|^2>) = mach_rms sqrt(gamma)."""
        n = self.n
        rng = np.random.default_rng(self.seed)
        w = rng.standard_normal((3, n, n, n))
        wh = np.fft.rfftn(w, axes=(1, 2, 3))
        del w
        kz = np.fft.fftfreq(n) * n
        ky = np.fft.fftfreq(n) * n
        kx = np.fft.rfftfreq(n) * n
        KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
        k2 = KX ** 2 + KY ** 2 + KZ ** 2
        k2[0, 0, 0] = 1.0
        # solenoidal projection u <- u - k (k.u) / |k|^2 (component order x, y, z)
        kdot = (KX * wh[0] + KY * wh[1] + KZ * wh[2]) / k2
        wh[0] -= KX * kdot
        wh[1] -= KY * kdot
        wh[2] -= KZ * kdot
        del kdot
        k = np.sqrt(k2)
        amp = np.sqrt(k ** 4 * np.exp(-2.0 * (k / 4.0) ** 2) / k2)
        amp[0, 0, 0] = 0.0
        wh *= amp[None]
        del amp, k, k2, KX, KY, KZ
        u = np.fft.irfftn(wh, s=(n, n, n), axes=(1, 2, 3))
        del wh
        rms = math.sqrt(float(np.mean(np.sum(u ** 2, axis=0))))
        u *= self.mach_rms * math.sqrt(self.gamma) / rms
        N = n ** 3
        # array index [z, y, x] flattens with x fastest
        return np.ones(N), u.reshape(3, N), np.ones(N)


def _trrs_fastest_speed(left, right, gamma):
    """Fastest wave speed of a shock tube, estimated with the two-rarefaction
    approximation of the star pressure (used only to size step counts)."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL = math.sqrt(gamma * pL / rL)
    cR = math.sqrt(gamma * pR / rR)
    z = (gamma - 1.0) / (2.0 * gamma)
    ps = ((cL + cR - 0.5 * (gamma - 1.0) * (uR - uL)) / (cL / pL ** z + cR / pR ** z)) ** (1.0 / z)
    sR = uR + cR * math.sqrt(max(1.0, (gamma + 1.0) / (2.0 * gamma) * ps / pR
                                 + (gamma - 1.0) / (2.0 * gamma)))
    sL = uL - cL * math.sqrt(max(1.0, (gamma + 1.0) / (2.0 * gamma) * ps / pL
                                 + (gamma - 1.0) / (2.0 * gamma)))
    return max(abs(sL), abs(sR))


@dataclass
class Batch:
    """Ragged batch of 1-D shock tubes, packed end to end.

    offsets[I+1] (int64): tube i owns nodes offsets[i] .. offsets[i+1]-1.
    Fields rho/u/T are packed the same way.  Per instance: gamma, n_rot, tau,
    steps (int64), left/right states."""
    lengths: np.ndarray
    offsets: np.ndarray
    gamma: np.ndarray
    n_rot: np.ndarray
    tau: np.ndarray
    steps: np.ndarray
    left: np.ndarray
    right: np.ndarray
    rho: np.ndarray = field(repr=False)
    u: np.ndarray = field(repr=False)
    T: np.ndarray = field(repr=False)

    @property
    def num(self):
        return len(self.lengths)

    @property
    def total(self):
        return int(self.offsets[-1])

    def subset(self, idx):
        idx = np.asarray(idx)
        parts = [slice(self.offsets[i], self.offsets[i + 1]) for i in idx]
        lengths = self.lengths[idx]
        return Batch(lengths, np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64),
                     self.gamma[idx], self.n_rot[idx], self.tau[idx], self.steps[idx],
                     self.left[idx], self.right[idx],
                     np.concatenate([self.rho[p] for p in parts]),
                     np.concatenate([self.u[:, p] for p in parts], axis=1),
                     np.concatenate([self.T[p] for p in parts]))


def batched_tubes(num=4096, seed=0, lmin=256, lmax=8192, gamma_range=(1.1, 1.67),
                  pr_range=(2.0, 100.0), dr_range=(1.0, 10.0), tau_range=(0.6, 1.0),
                  t_frac=0.8, fixed_length=None, r_lattice=R_PRINTED) -> Batch:
    """Shock tubes: L ~ round(exp U[ln lmin, ln lmax]) (or fixed_length),
    gamma ~ U[gamma_range], pressure ratio ~ logU[pr_range], density ratio ~
    U[dr_range], left (rho, u, p) = (1, 0, 1), right = (1/dr, 0, 1/pr),
    diaphragm at the midpoint, tau ~ U[tau_range], and
    steps = floor(t_frac * t_exit * L * r) with t_exit the time the fastest
    wave needs to reach an end of the unit-length tube."""
    rng = np.random.default_rng(seed)
    if fixed_length:
        lengths = np.full(num, int(fixed_length), dtype=np.int64)
    else:
        lengths = np.round(np.exp(rng.uniform(math.log(lmin), math.log(lmax), num))).astype(np.int64)
    gamma = rng.uniform(*gamma_range, num)
    pr = np.exp(rng.uniform(math.log(pr_range[0]), math.log(pr_range[1]), num))
    dr = rng.uniform(*dr_range, num)
    tau = rng.uniform(*tau_range, num)
    left = np.tile(np.array([1.0, 0.0, 1.0]), (num, 1))
    right = np.stack([1.0 / dr, np.zeros(num), 1.0 / pr], axis=1)
    steps = np.zeros(num, dtype=np.int64)
    for i in range(num):
        s = _trrs_fastest_speed(tuple(left[i]), tuple(right[i]), gamma[i])
        steps[i] = max(1, int(math.floor(t_frac * (0.5 / s) * lengths[i] * r_lattice)))
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    rho = np.empty(offsets[-1])
    u = np.zeros((1, offsets[-1]))
    T = np.empty(offsets[-1])
    for i in range(num):
        r_, u_, T_ = sod_tube(int(lengths[i]), left[i], right[i])
        sl = slice(offsets[i], offsets[i + 1])
        rho[sl], u[:, sl], T[sl] = r_, u_, T_
    return Batch(lengths, offsets, gamma, n_of_gamma(gamma, 1), tau, steps, left, right, rho, u, T)


def nonequilibrium_perturbation(shape, seed, amp=0.01):
    """Multiplicative factors 1 + amp*U(-1,1) used to push populations off
    equilibrium in parity tests."""
    return 1.0 + amp * np.random.default_rng(seed).uniform(-1.0, 1.0, shape)
