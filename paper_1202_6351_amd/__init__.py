"""MI355X (gfx950) implementation of the cascaded central-moment D2Q9 lattice
Boltzmann step (Ning & Premnath, Section II) with periodic, halfway
bounce-back and moving-wall boundaries (Section III), FP16/BF16 deviation
storage, and a hand-written adjoint for gradients.

The compute path is liblbm.so (include/lbm.h); this package only marshals
PyTorch tensors and streams to it.  Importing fails if the library is not
built.
"""
from . import _lib

_lib.lib()  # fail loudly at import if liblbm.so is missing

from .lattice import Lattice, Params, lattice_layout  # noqa: E402,F401
from .autograd import Rollout, rollout  # noqa: E402,F401

__all__ = ["Lattice", "Params", "lattice_layout", "Rollout", "rollout"]
