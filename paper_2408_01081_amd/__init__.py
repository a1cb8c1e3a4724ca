"""MI355X (gfx950) implementation of the vectorial lattice Boltzmann method for
2D linear elastodynamics (arXiv 2408.01081): HIP kernels behind a C ABI
(include/lbm.h) with a thin ctypes binding.  PyTorch supplies device memory
and streams only."""
from ._lib import LbmError, load  # noqa: F401

__all__ = ["LbmError", "load", "Lattice"]


def __getattr__(name):
    if name == "Lattice":
        from .lbm import Lattice
        return Lattice
    raise AttributeError(name)
