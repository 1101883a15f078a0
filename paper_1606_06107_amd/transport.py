"""Transport coefficients of the scheme measured on the GPU from decaying
Fourier modes on a periodic 2-D grid (lattice units: nodes, time steps).

shear_viscosity     a transverse velocity wave u_y = U sin(k x) decays as
                    exp(-nu k^2 t): nu.
thermal_diffusivity an isobaric temperature wave (rho T = const, u = 0)
                    decays as exp(-chi k^2 t) once the sound waves the
                    initial condition excites have been absorbed: chi.

The Chapman-Enskog analysis of the paper (Sec. II and the Appendix) gives
mu = (2/D) rho e_t tau and kappa = 2(D+n+2)/(D(D+n)) rho e_t tau for the
continuous equations; with the streaming step the lattice form is
nu = (T/r^2)(tau - 1/2).  The amplitudes are read as the Fourier coefficient
at k of the device fields; all arithmetic of the steps runs in the library."""
from __future__ import annotations

import math

import numpy as np
import torch

from .sim import Sim


def _amp(field, k, x):
    return 2.0 * abs(np.mean(field * np.exp(-1j * k * x)))


def _decay_rate(times, amps):
    return -np.polyfit(np.asarray(times, dtype=float), np.log(np.asarray(amps)), 1)[0]


def shear_viscosity(n_rot, tau, T0=1.0, nx=64, ny=3, U=0.01, every=100, samples=6,
                    dtype=torch.float64, lattice=None):
    """nu (nodes^2 per step) from the decay of u_y = U sin(2 pi x / nx)."""
    N = nx * ny
    x = np.tile(np.arange(nx), ny)
    k = 2 * math.pi / nx
    u = np.zeros((2, N))
    u[1] = U * np.sin(k * x)
    sim = Sim((nx, ny), n_rot=n_rot, tau=tau, dtype=dtype, lattice=lattice).init(np.ones(N), u, np.full(N, T0))
    t, a = [], []
    for s in range(samples):
        sim.step(every)
        t.append(every * (s + 1))
        a.append(_amp(sim.moments(totals=False)[1][1].cpu().numpy(), k, x))
    return _decay_rate(t, a) / k ** 2


def thermal_diffusivity(n_rot, tau, T0=1.0, nx=64, ny=3, eps=0.01, every=100, samples=6, skip=2,
                        dtype=torch.float64, lattice=None):
    """chi (nodes^2 per step) from the decay of T = T0 (1 + eps sin(2 pi x / nx))
    at constant pressure; the first `skip` samples (acoustic transient) are
    left out of the fit."""
    N = nx * ny
    x = np.tile(np.arange(nx), ny)
    k = 2 * math.pi / nx
    s_ = np.sin(k * x)
    sim = Sim((nx, ny), n_rot=n_rot, tau=tau, dtype=dtype, lattice=lattice)
    sim.init(1.0 / (1 + eps * s_), np.zeros((2, N)), T0 * (1 + eps * s_))
    t, a = [], []
    for s in range(samples):
        sim.step(every)
        t.append(every * (s + 1))
        a.append(_amp(sim.moments(totals=False)[2].cpu().numpy(), k, x))
    return _decay_rate(t[skip:], a[skip:]) / k ** 2
