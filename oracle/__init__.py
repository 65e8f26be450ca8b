"""FP64 CPU oracle of the cascaded (central-moment MRT) D2Q9 LBM.

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU library is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product package never does, and this package
imports nothing from the product.

`oracle/lbmref.c` follows the paper's Section II explicit formulas (raw moments
of f-bar, source moments, collision kernels g3..g8, post-collision
populations) and the Section III boundary treatments.  `oracle/ref_torch.py`
is an independent plain-definition formulation in float64 PyTorch (dense 9x9
central-moment matrices and a linear solve), used as the autograd gradient
reference on tiny grids.
"""
from .lbmref import (  # noqa: F401
    Params,
    build,
    collide,
    diagnostics,
    equilibrium,
    init_state,
    kmatrix,
    library_path,
    macroscopic,
    num_threads,
    source,
    step,
    step_at,
)
