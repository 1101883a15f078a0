"""ctypes binding of liblbmx.so (the C ABI in include/lbm.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Loading fails loudly if the library has not been built; there is no
CPU fallback."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LBMX_LIB names another build of the same sources (the host-sanitizer build
# of the test suite's address/undefined-behaviour check).
LIB_PATH = os.environ.get("LBMX_LIB") or os.path.join(HERE, "liblbmx.so")

LBM_ABI_VERSION = 2
LBM_OK, LBM_EINVAL, LBM_EDEVICE, LBM_ENOMEM, LBM_EUNSUPPORTED, LBM_ELAUNCH = range(6)
LBM_D1Q7, LBM_D2Q49, LBM_D3Q343, LBM_D2Q37 = 1, 2, 3, 4
LBM_F32, LBM_F64 = 0, 1
LBM_BC_PERIODIC, LBM_BC_OPEN = 0, 1
LBM_DEBUG_POISON = 1

c_i32, c_i64, c_dbl, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class LbmDesc(ctypes.Structure):
    _fields_ = [("abi_version", c_i32), ("dim", c_i32), ("n", c_i64 * 3), ("lattice", c_i32),
                ("dtype", c_i32), ("bc", c_i32 * 3), ("n_rot", c_dbl), ("tau", c_dbl),
                ("g_substeps", c_i32), ("f", c_vp * 2), ("g", c_vp * 2), ("workspace", c_vp)]


class LbmBatchDesc(ctypes.Structure):
    _fields_ = [("abi_version", c_i32), ("dtype", c_i32), ("num_instances", c_i64),
                ("total_nodes", c_i64), ("offsets", c_vp), ("n_rot", c_vp), ("tau", c_vp),
                ("nsteps", c_vp), ("f", c_vp * 2), ("g", c_vp * 2), ("status", c_vp),
                ("steps_done", c_vp),
                ("workspace", c_vp), ("block", c_i32), ("chunk", c_i32), ("superstep", c_i32),
                ("g_substeps", c_i32)]


class LbmSurDesc(ctypes.Structure):
    _fields_ = [("abi_version", c_i32), ("batch", c_i32), ("length", c_i32), ("params", c_vp),
                ("params_bf16", c_vp), ("workspace", c_vp)]


LBM_SUR_NPARAMS = 69708
LBM_SUR_K = 16

# name -> (restype, argtypes); every symbol include/lbm.h declares
SIGNATURES = {
    "lbm_workspace_bytes": (c_sz, [ctypes.POINTER(LbmDesc)]),
    "lbm_init": (c_i32, [ctypes.POINTER(LbmDesc), c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(c_vp)]),
    "lbm_init_populations": (c_i32, [ctypes.POINTER(LbmDesc), c_vp, c_vp, c_vp, ctypes.POINTER(c_vp)]),
    "lbm_step": (c_i32, [c_vp, c_i64]),
    "lbm_prepare": (c_i32, [c_vp, c_i64]),
    "lbm_moments": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lbm_populations": (c_i32, [c_vp, c_vp, c_vp]),
    "lbm_set_monitor": (c_i32, [c_vp, c_i64, c_vp, c_i64]),
    "lbm_time": (c_i32, [c_vp, ctypes.POINTER(c_i64)]),
    "lbm_set_graphs": (c_i32, [c_vp, c_i32]),
    "lbm_set_debug": (c_i32, [c_vp, c_i32]),
    "lbm_set_tile": (c_i32, [c_vp, c_i32, c_i32, c_i32]),
    "lbm_set_inplace": (c_i32, [c_vp, c_i32]),
    "lbm_set_blocked": (c_i32, [c_vp, c_i32]),
    "lbm_set_fd": (c_i32, [c_vp, ctypes.c_double]),
    "lbm_destroy": (c_i32, [c_vp]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_stream_copy": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
    "lbm_pattern_probe": (c_i32, [c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_i32, c_i32, c_vp]),
    "lbm_pattern_probe_3d": (c_i32, [c_i32, c_vp, c_vp, c_vp, c_vp, c_i32, c_i32, c_i32, c_vp]),
    "lbm_lattice_info": (c_i32, [c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_dbl), c_vp, c_vp]),
    "lbm_batch_workspace_bytes": (c_sz, [ctypes.POINTER(LbmBatchDesc)]),
    "lbm_batch_init": (c_i32, [ctypes.POINTER(LbmBatchDesc), c_vp, c_vp, c_vp, c_vp]),
    "lbm_batch_step": (c_i32, [ctypes.POINTER(LbmBatchDesc), c_vp]),
    "lbm_batch_step_noalloc": (c_i32, [ctypes.POINTER(LbmBatchDesc), c_vp]),
    "lbm_batch_release": (c_i32, [ctypes.POINTER(LbmBatchDesc)]),
    "lbm_batch_moments": (c_i32, [ctypes.POINTER(LbmBatchDesc), c_vp, c_vp, c_vp, c_vp]),
    "lbm_sur_bf16_bytes": (c_sz, []),
    "lbm_sur_workspace_bytes": (c_sz, [ctypes.POINTER(LbmSurDesc)]),
    "lbm_sur_pack": (c_i32, [ctypes.POINTER(LbmSurDesc), c_vp]),
    "lbm_sur_forward": (c_i32, [ctypes.POINTER(LbmSurDesc), c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lbm_sur_backward": (c_i32, [ctypes.POINTER(LbmSurDesc), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lbm_sur_adam": (c_i32, [ctypes.POINTER(LbmSurDesc), c_vp, c_vp, c_vp, c_vp, ctypes.c_float,
                             ctypes.c_float, ctypes.c_float, ctypes.c_float, c_i64, c_vp]),
    "lbm_sur_check": (c_i32, [ctypes.POINTER(LbmSurDesc), c_vp, c_vp, c_vp, c_dbl, c_dbl, c_dbl, c_dbl,
                              c_vp, c_vp]),
    "lbm_sur_lift": (c_i32, [ctypes.POINTER(LbmSurDesc), c_vp, c_vp, c_vp, ctypes.POINTER(LbmBatchDesc), c_i64,
                             c_vp]),
    "lbm_sur_merge": (c_i32, [ctypes.POINTER(LbmSurDesc), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
}

_lib = None


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"liblbmx status {status}: {msg}")
        self.status = status


def load():
    """Load liblbmx.so (built by __graft_entry__.build()).  Raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int):
    if status != LBM_OK:
        raise LbmError(status, load().lbm_last_error().decode())
    return status
