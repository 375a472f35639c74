"""MI355X (gfx950) matrix-free solver for the 3D heterogeneous Helmholtz equation.

CSLP-preconditioned Bi-CGSTAB on the 7-point operator, the preconditioner
inverted by one geometric multigrid V-cycle (Chen, Dwarka, Vuik, arXiv
2308.06085), as hand-written HIP kernels behind the C ABI of include/hh.h.
"""
from .solver import HelmholtzSolve, SolveStats, Solver  # noqa: F401

__all__ = ["Solver", "SolveStats", "HelmholtzSolve"]
