"""MI355X-native tensor-product multigrid for the anisotropic Helmholtz-type
pressure equation on a latitude-longitude shell (arXiv 2307.04528).

The solver (setup, V-cycles, FP64 refinement, adjoint) runs in the HIP
library libmgshell.so built from ``csrc/`` (see ``build.py``); this package is
its Python binding. Importing it does not load the library; the first call
does, and fails loudly if the library is missing.
"""
from .solver import Solver, SolveStats, mg_plan, mg_plan_tables
from .autograd import MGSolve, mg_solve

__all__ = ["Solver", "SolveStats", "MGSolve", "mg_solve", "mg_plan", "mg_plan_tables"]
