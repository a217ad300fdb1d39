"""CPU oracle for the Wilson-Dirac conjugate-gradient solve -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct FP64 numpy code that states what the GPU
library computes. Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import it; the library's own code path
never does (there is no CPU fallback).

It shares no code with the HIP path: no kernels, headers, tables or helpers.
The only common code is ``fieldgen`` (seeded inputs; none of the method's
arithmetic).

Modules
  dirac   -- gamma matrices, the Wilson-Dirac operator D and its adjoint,
             dense assembly for tiny lattices, site-local evaluation.
  solver  -- conjugate gradient on the normal equations (CGNR), dense solve.
  force   -- derivative of the solve with respect to the gauge links.
  laplace -- a second operator through the same CG: the gauge-covariant
             lattice Laplacian on colour vectors, plain CG, dense assembly.

Parity status: every function here is pinned by the ``-m "not gpu"`` tests
in ``tests/test_oracle_*.py`` against closed forms, invariants and brute
force (free-field momentum-space spectrum, plane waves, gamma_5
hermiticity, gauge covariance, dense direct solves, finite differences).
"""
from .dirac import (
    GAMMA,
    GAMMA5,
    wilson_D,
    wilson_Ddag,
    normal_op,
    dense_D,
    wilson_D_sites,
    normal_op_sites,
    site_index,
)
from .solver import cgnr, dense_solve_normal, true_relative_residual
from .force import force_G, solve_gradients
from . import laplace

__all__ = [
    "GAMMA",
    "GAMMA5",
    "wilson_D",
    "wilson_Ddag",
    "normal_op",
    "dense_D",
    "wilson_D_sites",
    "normal_op_sites",
    "site_index",
    "cgnr",
    "dense_solve_normal",
    "true_relative_residual",
    "force_G",
    "solve_gradients",
    "laplace",
]
