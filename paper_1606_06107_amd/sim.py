"""Python front end of the per-step simulator (lbm_init / lbm_step /
lbm_moments / lbm_populations).  PyTorch provides device memory and the
stream; the library's kernels do the work."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

_LATTICE = {1: L.LBM_D1Q7, 2: L.LBM_D2Q49, 3: L.LBM_D3Q343}
_Q = {1: 7, 2: 49, 3: 343}
_NAMED = {"D1Q7": (1, L.LBM_D1Q7, 7), "D2Q49": (2, L.LBM_D2Q49, 49), "D2Q37": (2, L.LBM_D2Q37, 37),
          "D3Q343": (3, L.LBM_D3Q343, 343)}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def lattice_info(dim_or_name):
    """(Q, r, w[Q], c[Q,3]) as the library computes with them, by dimension
    (tensor lattices) or name ("D2Q37", ...); rows in storage-slot order."""
    import numpy as np
    lib = L.load()
    Q = ctypes.c_int32()
    r = ctypes.c_double()
    if isinstance(dim_or_name, str):
        _, lat, q = _NAMED[dim_or_name]
    else:
        lat, q = _LATTICE[dim_or_name], _Q[dim_or_name]
    w = np.zeros(q)
    c = np.zeros((q, 3), dtype=np.int32)
    L.check(lib.lbm_lattice_info(lat, ctypes.byref(Q), ctypes.byref(r),
                                 w.ctypes.data_as(ctypes.c_void_p), c.ctypes.data_as(ctypes.c_void_p)))
    return Q.value, r.value, w, c


class Sim:
    """A grid of nodes on one GPU.  Tile, graph, streaming-scheme and
    population-order settings persist across init / init_populations (each
    creates a new handle).

    shape: nodes per axis (x first), bc: 'periodic' | 'open' per axis,
    n_rot: rotational degrees of freedom (gamma = (D+n+2)/(D+n)), tau: BGK
    relaxation time in steps, dtype: torch.float32 | torch.float64, lattice:
    None (D1Q7^D) or "D2Q37" (2-D, Table I), g_substeps: 1 = the rotational
    update as the paper writes it, m > 1 = its advection in m sub-steps
    (lbm_desc.g_substeps)."""

    def __init__(self, shape, bc=None, n_rot=0.0, tau=1.0, dtype=torch.float32,
                 device="cuda", stream=None, lattice=None, g_substeps=1):
        self.lib = L.load()
        shape = tuple(int(s) for s in shape)
        self.D = len(shape)
        assert 1 <= self.D <= 3
        self.shape = shape
        self.N = 1
        for s in shape:
            self.N *= s
        if lattice is None:
            self.lattice, self.Q = _LATTICE[self.D], _Q[self.D]
        else:
            dim, self.lattice, self.Q = _NAMED[lattice]
            assert dim == self.D, f"{lattice} needs a {dim}-D grid"
        bc = bc or ["periodic"] * self.D
        self.dtype = dtype
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.f = [torch.empty((self.Q, self.N), dtype=dtype, device=self.device) for _ in range(2)]
        self.g = [torch.empty((7, self.N), dtype=dtype, device=self.device) for _ in range(2)]
        d = L.LbmDesc()
        d.abi_version = L.LBM_ABI_VERSION
        d.dim = self.D
        n = list(shape) + [1] * (3 - self.D)
        for a in range(3):
            d.n[a] = n[a]
            d.bc[a] = L.LBM_BC_OPEN if (a < self.D and bc[a] == "open") else L.LBM_BC_PERIODIC
        d.lattice = self.lattice
        d.dtype = L.LBM_F32 if dtype == torch.float32 else L.LBM_F64
        d.n_rot = float(n_rot)
        d.tau = float(tau)
        d.g_substeps = int(g_substeps)
        for k in range(2):
            d.f[k] = self.f[k].data_ptr()
            d.g[k] = self.g[k].data_ptr()
        nbytes = self.lib.lbm_workspace_bytes(ctypes.byref(d))
        self.workspace = torch.empty(max(nbytes, 256) // 8, dtype=torch.float64, device=self.device)
        d.workspace = self.workspace.data_ptr()
        self.desc = d
        self.handle = None
        self.n_rot, self.tau = float(n_rot), float(tau)
        # settings re-applied to every new handle (init / init_populations)
        self._tile = None
        self._graphs = None
        self._inplace = None
        self._blocked = None
        self._fd = None
        self._debug = None

    def _apply_settings(self):
        if self._fd is not None:  # first: it decides the streaming scheme
            L.check(self.lib.lbm_set_fd(self.handle, float(self._fd)))
        if self._blocked is not None:  # first: enabling it resets the tile
            L.check(self.lib.lbm_set_blocked(self.handle, 1 if self._blocked else 0))
        if self._tile is not None:
            L.check(self.lib.lbm_set_tile(self.handle, *[int(v) for v in self._tile]))
        if self._graphs is not None:
            L.check(self.lib.lbm_set_graphs(self.handle, 1 if self._graphs else 0))
        if self._inplace is not None:
            L.check(self.lib.lbm_set_inplace(self.handle, 1 if self._inplace else 0))
        if self._debug is not None:
            L.check(self.lib.lbm_set_debug(self.handle, L.LBM_DEBUG_POISON if self._debug else 0))

    def _stream_ptr(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def init(self, rho, u, T):
        """Equilibrium initial state from FP64 fields rho[N], u[D,N], T[N]
        (numpy or torch; copied to the device)."""
        dev = self.device
        self._fields = [torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
                        for a in (rho, u, T)]
        rho_t, u_t, T_t = self._fields
        assert rho_t.numel() == self.N and u_t.numel() == self.D * self.N and T_t.numel() == self.N
        self.stream.wait_stream(torch.cuda.current_stream(dev))  # conversions above ran there
        self._free()
        h = ctypes.c_void_p()
        with torch.cuda.stream(self.stream):
            L.check(self.lib.lbm_init(ctypes.byref(self.desc), _ptr(rho_t), _ptr(u_t), _ptr(T_t),
                                      self._stream_ptr(), ctypes.byref(h)))
        self.handle = h
        self._apply_settings()
        return self

    def init_populations(self, f0, g0):
        f0 = torch.as_tensor(f0).to(self.device, self.dtype).contiguous()
        g0 = torch.as_tensor(g0).to(self.device, self.dtype).contiguous()
        assert f0.shape == (self.Q, self.N) and g0.shape == (7, self.N)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))  # conversions above ran there
        self._keep = (f0, g0)
        self._free()
        h = ctypes.c_void_p()
        L.check(self.lib.lbm_init_populations(ctypes.byref(self.desc), _ptr(f0), _ptr(g0),
                                              self._stream_ptr(), ctypes.byref(h)))
        self.handle = h
        self._apply_settings()
        return self

    def step(self, nsteps=1):
        L.check(self.lib.lbm_step(self.handle, int(nsteps)))
        return self

    def prepare(self, nsteps):
        """Record and instantiate the HIP graph of step(nsteps) from the
        current state without running it (host work done ahead of a timed
        or latency-critical call)."""
        L.check(self.lib.lbm_prepare(self.handle, int(nsteps)))
        return self

    def set_debug(self, poison: bool):
        """Poison every step's write-only destinations with NaN first, so that
        a value a step fails to write shows up (lbm_set_debug)."""
        L.check(self.lib.lbm_set_debug(self.handle, L.LBM_DEBUG_POISON if poison else 0))
        self._debug = bool(poison)
        return self

    def set_graphs(self, on: bool):
        L.check(self.lib.lbm_set_graphs(self.handle, 1 if on else 0))
        self._graphs = bool(on)

    def set_inplace(self, on: bool):
        """Translational streaming in one buffer (True) or ping-pong (False);
        only before the first step.  Default: in place on fully periodic 1-D/2-D
        grids."""
        L.check(self.lib.lbm_set_inplace(self.handle, 1 if on else 0))
        self._inplace = bool(on)
        return self

    def set_fd(self, courant: float):
        """Finite-difference update of Sec. V A for f as well (courant in
        (0, 1]: time step courant * dx / r), or collide-and-stream (0, the
        default); only before the first step.  1-D and 2-D grids."""
        L.check(self.lib.lbm_set_fd(self.handle, float(courant)))
        self._fd = float(courant)
        return self

    def set_blocked(self, on: bool):
        """3-D only: populations in blocks of 64 x-consecutive nodes (True) or
        plain [Q][N] (False); only before the first step.  Default: blocked
        when n0 is a multiple of 64.  Enabling sets the tile to 64x1x1."""
        L.check(self.lib.lbm_set_blocked(self.handle, 1 if on else 0))
        self._blocked = bool(on)
        if on:
            self._tile = None
        return self

    def set_tile(self, tx, ty=1, tz=1):
        L.check(self.lib.lbm_set_tile(self.handle, int(tx), int(ty), int(tz)))
        self._tile = (int(tx), int(ty), int(tz))

    def set_monitor(self, every, capacity):
        """Record totals every `every` steps into a device tensor [capacity, 2+D]."""
        self.series = torch.full((int(capacity), 2 + self.D), float("nan"), dtype=torch.float64,
                                 device=self.device)
        L.check(self.lib.lbm_set_monitor(self.handle, int(every), _ptr(self.series), int(capacity)))
        return self.series

    @property
    def t(self):
        v = ctypes.c_int64()
        L.check(self.lib.lbm_time(self.handle, ctypes.byref(v)))
        return v.value

    def moments(self, fields=True, totals=True):
        """(rho[N], u[D,N], T[N], totals[2+D]) as FP64 device tensors."""
        dev = self.device
        rho = torch.empty(self.N, dtype=torch.float64, device=dev) if fields else None
        u = torch.empty((self.D, self.N), dtype=torch.float64, device=dev) if fields else None
        T = torch.empty(self.N, dtype=torch.float64, device=dev) if fields else None
        tot = torch.empty(2 + self.D, dtype=torch.float64, device=dev) if totals else None
        L.check(self.lib.lbm_moments(self.handle, _ptr(rho), _ptr(u), _ptr(T), _ptr(tot)))
        return rho, u, T, tot

    def populations(self):
        """Streamed f(t) [Q,N] and g(t) [7,N] as device tensors."""
        f = torch.empty((self.Q, self.N), dtype=self.dtype, device=self.device)
        g = torch.empty((7, self.N), dtype=self.dtype, device=self.device)
        L.check(self.lib.lbm_populations(self.handle, _ptr(f), _ptr(g)))
        return f, g

    def _free(self):
        if self.handle is not None:
            self.lib.lbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self._free()
        except Exception:
            pass
