"""MI355X (gfx950) implementation of the decoupled Hermite-expansion lattice
Boltzmann scheme for compressible flow with arbitrary specific heat ratio
(Hu, Zhang & Geng, arXiv:1606.06107).

The numerical work runs in the HIP kernels of liblbmx.so behind the C ABI of
include/lbm.h; this package only marshals arguments (PyTorch supplies device
memory and streams).  Importing the package does not load the library; the
first use does, and fails loudly if it has not been built.
"""
from ._lib import LbmError, load  # noqa: F401

__all__ = ["LbmError", "load", "Sim", "Batch", "Surrogate", "lattice_info"]


def __getattr__(name):
    if name in ("Sim", "lattice_info"):
        from . import sim
        return getattr(sim, name)
    if name == "Batch":
        from . import batch
        return batch.Batch
    if name == "Surrogate":
        from . import surrogate
        return surrogate.Surrogate
    raise AttributeError(name)
