"""CPU oracle for the CSLP-preconditioned Bi-CGSTAB Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex128 NumPy /
SciPy implementation of what the solver computes, written from the paper
(Chen, Dwarka, Vuik, "A matrix-free parallel solution method for the
three-dimensional heterogeneous Helmholtz equation", arXiv 2308.06085).
Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the GPU library and never imports it.

Modules
-------
``discretization``  grid, 7-point operators A_h and M_h with Sommerfeld ghost
                    elimination, Dirac right-hand side, closed-off problem
                    (paper section 2.1, 2.4; section 3.3; Algorithm 2).
``multigrid``       damped Jacobi, full weighting, trilinear interpolation,
                    rediscretised coarse operators, exact coarsest solve,
                    recursive V- and F-cycles (section 3.4, Algorithm 1,
                    section 4.2).
``krylov``          right-preconditioned Bi-CGSTAB and IDR(s) with the
                    true-residual stopping rule of section 5; left-preconditioned
                    full GMRES with the preconditioned-residual rule.
``adjoint``         misfit gradient with respect to squared slowness by one
                    adjoint solve.

Every function is pinned by the ``-m "not gpu"`` tests against closed forms,
invariants, library routines or the paper's printed iteration counts; the
one exception is listed as "parity unpinned" in ``adjoint`` (none at present).
"""
from .discretization import (  # noqa: F401
    Level,
    boundary_directions,
    apply_operator,
    apply_A,
    apply_M,
    diag_M,
    point_source_rhs,
    closed_off_problem,
    unknown_mask,
)
from .multigrid import (  # noqa: F401
    Hierarchy,
    build_hierarchy,
    jacobi_sweep,
    restrict_fw,
    prolong_trilinear,
    vcycle,
    fcycle,
)
from .krylov import bicgstab, gmres, idrs, SolveResult, Status  # noqa: F401
from .adjoint import misfit_and_gradient, adjoint_gradient_pointwise, solve_forward  # noqa: F401
