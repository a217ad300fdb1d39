"""MI355X (gfx950) Wilson-Dirac conjugate-gradient library.

The computation lives in the HIP shared library libwilson_mi355x.so (C ABI
in include/wilson.h); this package only marshals tensors into it. Build with
``python -m paper_2001_05218_amd.build``.
"""
from ._lib import load, last_error, WilsonError  # noqa: F401
from .ops import (  # noqa: F401
    wilson_apply,
    wilson_force,
    cg_solve,
    cg_solve_batched,
    cg_solve_ooc,
    ooc_workspace_bytes,
    pack_gauge,
    pack_spinor,
    unpack_spinor,
    empty_packed_spinor,
    wilson_apply_packed,
    workspace_bytes,
    laplace_apply,
    laplace_cg_solve,
    laplace_workspace_bytes,
)
from .autograd import WilsonSolve, wilson_solve  # noqa: F401
