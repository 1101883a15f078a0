"""Python front end of the batched shock tubes (lbm_batch_init /
lbm_batch_step / lbm_batch_moments): many independent 1-D D1Q7 + D1Q7 tubes
of uneven length, per-instance n, tau and step count, advanced by one
persistent launch.  PyTorch provides device memory and the stream."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Batch:
    """lengths[I] (>= 1 each), n_rot[I], tau[I], nsteps[I] (per call of
    step()).  block/chunk/superstep: launch shape (0 = library default;
    chosen by the autotuner).  g_substeps: rotational advection sub-steps
    per step (1 = the update as written; lbm_batch_desc.g_substeps)."""

    def __init__(self, lengths, n_rot, tau, nsteps, dtype=torch.float32, device="cuda",
                 block=0, chunk=0, superstep=0, stream=None, g_substeps=1):
        self.lib = L.load()
        dev = torch.device(device)
        lengths = np.asarray(lengths, dtype=np.int64)
        self.I = len(lengths)
        self.offsets_h = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
        self.total = int(self.offsets_h[-1])
        self.dtype, self.device = dtype, dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.offsets = torch.as_tensor(self.offsets_h, device=dev)
        self.n_rot = torch.as_tensor(np.asarray(n_rot, dtype=np.float64), device=dev)
        self.tau = torch.as_tensor(np.asarray(tau, dtype=np.float64), device=dev)
        self.nsteps = torch.as_tensor(np.asarray(nsteps, dtype=np.int64), device=dev)
        self.f = [torch.empty((7, self.total), dtype=dtype, device=dev) for _ in range(2)]
        self.g = [torch.empty((7, self.total), dtype=dtype, device=dev) for _ in range(2)]
        self.status = torch.full((self.I,), -1, dtype=torch.int32, device=dev)
        self.steps_done = torch.zeros((self.I,), dtype=torch.int64, device=dev)
        d = L.LbmBatchDesc()
        d.abi_version = L.LBM_ABI_VERSION
        d.dtype = L.LBM_F32 if dtype == torch.float32 else L.LBM_F64
        d.num_instances = self.I
        d.total_nodes = self.total
        d.offsets = self.offsets.data_ptr()
        d.n_rot = self.n_rot.data_ptr()
        d.tau = self.tau.data_ptr()
        d.nsteps = self.nsteps.data_ptr()
        for k in range(2):
            d.f[k] = self.f[k].data_ptr()
            d.g[k] = self.g[k].data_ptr()
        d.status = self.status.data_ptr()
        d.steps_done = self.steps_done.data_ptr()
        d.block, d.chunk, d.superstep = int(block), int(chunk), int(superstep)
        d.g_substeps = int(g_substeps)
        nbytes = self.lib.lbm_batch_workspace_bytes(ctypes.byref(d))
        self.workspace = torch.empty(max(nbytes, 256) // 4 + 64, dtype=torch.int32, device=dev)
        d.workspace = self.workspace.data_ptr()
        self.desc = d

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def init(self, rho, u, T):
        """Equilibrium initial state from packed FP64 fields (length total;
        numpy arrays or torch tensors, device tensors used in place)."""
        self._fields = [torch.as_tensor(a, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
                        for a in (rho, u, T)]
        self.stream.wait_stream(torch.cuda.current_stream(self.device))  # conversions above ran there
        r, u_, T_ = self._fields
        assert r.numel() == self.total and u_.numel() == self.total and T_.numel() == self.total
        L.check(self.lib.lbm_batch_init(ctypes.byref(self.desc), _p(r), _p(u_), _p(T_), self._s()))
        return self

    def set_nsteps(self, nsteps):
        """Steps of the next call per tube (copied on the batch's stream, after
        the work already queued there)."""
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            self.nsteps.copy_(torch.as_tensor(np.asarray(nsteps, dtype=np.int64)))
        cur.wait_stream(self.stream)

    def step(self, stream=None, chunk=None, superstep=None):
        """Advance every tube i by nsteps[i] steps (one persistent launch), on
        the batch's stream or on `stream`; `chunk` and `superstep` override the
        batch's launch shape for this call (0: the library's default)."""
        s = self._s() if stream is None else ctypes.c_void_p(stream.cuda_stream)
        keep = self.desc.chunk, self.desc.superstep
        if chunk is not None:
            self.desc.chunk = int(chunk)
        if superstep is not None:
            self.desc.superstep = int(superstep)
        try:
            L.check(self.lib.lbm_batch_step(ctypes.byref(self.desc), s))
        finally:
            self.desc.chunk, self.desc.superstep = keep
        return self

    def step_noalloc(self):
        """step() through lbm_batch_step_noalloc: the library's fixed device
        scratch instead of this batch's workspace, direct launches, no
        allocation.  Same results."""
        L.check(self.lib.lbm_batch_step_noalloc(ctypes.byref(self.desc), self._s()))
        return self

    def moments(self):
        """Packed FP64 (rho, u, T) device tensors of the current state."""
        dev = self.device
        r = torch.empty(self.total, dtype=torch.float64, device=dev)
        u = torch.empty(self.total, dtype=torch.float64, device=dev)
        T = torch.empty(self.total, dtype=torch.float64, device=dev)
        L.check(self.lib.lbm_batch_moments(ctypes.byref(self.desc), _p(r), _p(u), _p(T), self._s()))
        return r, u, T

    def release(self):
        """Drop the library's HIP graph for this batch (its buffers are about
        to be freed); a later step() records a new one."""
        if getattr(self, "desc", None) is not None:
            L.check(self.lib.lbm_batch_release(ctypes.byref(self.desc)))

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def split(self, packed):
        """Host list of per-tube arrays from a packed device or host array."""
        a = packed.cpu().numpy() if torch.is_tensor(packed) else np.asarray(packed)
        return [a[..., self.offsets_h[i]:self.offsets_h[i + 1]] for i in range(self.I)]
