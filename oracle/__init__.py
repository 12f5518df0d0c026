"""Oracle: a plain, slow FP64 CPU implementation of the tensor-product multigrid
solve of the anisotropic Helmholtz-type pressure equation on a lat-lon shell.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import anything from this package. It shares no
code with the HIP path (kernels, host setup, C ABI or Python binding) and never
imports it; the only common module is ``shellgen`` (seeded random inputs).

What it follows (the paper, arXiv 2307.04528):
  * Section 2: the problem Hu = b with H a sparse Laplacian-like matrix; the
    multigrid V-cycle (smooth, restrict the residual, solve the coarse
    equation, prolongate, smooth again) and the residual norm ||b - Hu||.
  * Section 2.1, Eq. (1): the split H = H_z + dH and the stationary
    block-Jacobi (vertical line) iteration used as the smoother; horizontal-
    only coarsening.
  * Section 2.2: conditional semi-coarsening driven by the per-latitude
    horizontal anisotropy.
  * Section 2.3: a shallow hierarchy with a simple iterative method on the
    coarsest grid.
Where the paper is silent (discretisation, transfer operators, omega, the
anisotropy threshold, the coarse solver), the module docstrings state the
reading taken.

Parity status: every function is pinned by tests under ``tests/`` against
closed forms, library routines, exact rational arithmetic or invariants, except
where a docstring says "parity unpinned".
"""
from .geometry import vertical_coords, fine_lat_edges, Level
from .hierarchy import build_hierarchy, coarsen_rows, anisotropy
from .operator import apply, mtilde, assemble, column_pivots, column_solve
from .multigrid import (Options, sweep, sweep_from_zero, restrict, prolong,
                        prolong_T, inject, prolong_weights,
                        vcycle, vcycle_T, solve, solve_adjoint,
                        grad_alpha, cell_volumes, convergence_factors, sweep_omegas)

__all__ = [
    "vertical_coords", "fine_lat_edges", "Level", "build_hierarchy",
    "coarsen_rows", "anisotropy", "apply", "mtilde", "assemble",
    "column_pivots", "column_solve", "Options", "sweep", "sweep_from_zero",
    "restrict", "prolong", "prolong_T", "inject", "prolong_weights", "vcycle", "vcycle_T", "solve", "solve_adjoint",
    "grad_alpha", "cell_volumes", "convergence_factors", "sweep_omegas",
]
