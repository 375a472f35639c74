"""Misfit gradient with respect to squared slowness (oracle; test infrastructure only).

Forward model: A(s) u = b with k = omega sqrt(s) (paper section 2,
k = 2 pi f / c; s = 1/c^2 is the squared slowness), A(s) the Sommerfeld
operator of section 2.4.  Loss L = 1/2 ||R u - d||^2 with R the sampling at
receiver nodes.

Derivation (the paper has no adjoint; this is the standard discrete one):
* only the diagonal of A depends on s:
      A_jj = 6/h^2 - omega^2 s_j - n_j 2 i omega sqrt(s_j) / h,
  so a'_j = dA_jj/ds_j = -omega^2 - i n_j omega / (h sqrt(s_j)),
  with n_j the number of faces node j lies on (the boundary term is kept:
  the finite differences see the full discrete A(s));
* with g = R^T (R u - d) (the gradient of L with respect to u in the
  conjugate-Wirtinger convention that PyTorch uses),
      dL/ds_j = -Re( conj(lam_j) a'_j u_j ),   A^H lam = g;
* ghost elimination makes A non-symmetric, but D A is complex symmetric with
  D_j = 2^(-n_j) (the mirror coupling is doubled on each face).  Hence
  A^T = D A D^-1 and A^H lam = g  <=>  A w = D^-1 conj(g) with conj(lam) = D w:
  the adjoint needs one more solve with the same operator and preconditioner,
      dL/ds_j = -Re( D_j w_j a'_j u_j ).
"""
from __future__ import annotations

import numpy as np

from .discretization import Level, SOMMERFELD, apply_A, boundary_directions, point_source_rhs
from .krylov import bicgstab
from .multigrid import build_hierarchy, vcycle


def _level(s, omega, h):
    return Level(s.shape, h, omega * np.sqrt(s), SOMMERFELD)


def solve_forward(s, omega, h, rhs, tol=1e-10, maxit=2000):
    """u = A(s)^{-1} rhs with the CSLP-preconditioned Bi-CGSTAB of ``krylov``."""
    lvl = _level(s, omega, h)
    hier = build_hierarchy(lvl.k, h, SOMMERFELD)
    res = bicgstab(lambda x: apply_A(x, lvl), lambda r: vcycle(r, hier), rhs, tol=tol,
                   maxit=maxit)
    return res


def sample(u, receivers):
    return np.array([u[n] for n in receivers])


def adjoint_gradient_pointwise(u, w, s, omega, h):
    """grad_j = -Re(D_j w_j a'_j u_j), D_j = 2^(-n_j), a'_j = -omega^2 - i n_j omega / (h sqrt(s_j))."""
    nj = boundary_directions(s.shape)
    a_prime = -omega**2 - 1j * nj * omega / (h * np.sqrt(s))
    d = 2.0 ** (-nj)
    return -np.real(d * w * a_prime * u)


def adjoint_rhs(g, shape):
    """D^{-1} conj(g) with D_j = 2^(-n_j)."""
    nj = boundary_directions(shape)
    return (2.0 ** nj) * np.conj(g)


def misfit_and_gradient(s, omega, h, source, receivers, d, tol=1e-10):
    """Return (L, dL/ds, u) for L = 1/2 ||R u(s) - d||^2."""
    b = point_source_rhs(s.shape, h, [source])[0]
    u = solve_forward(s, omega, h, b, tol).x
    resid = sample(u, receivers) - d
    loss = 0.5 * float(np.sum(np.abs(resid) ** 2))
    g = np.zeros_like(u)
    for val, node in zip(resid, receivers):
        g[node] += val
    w = solve_forward(s, omega, h, adjoint_rhs(g, s.shape), tol).x
    return loss, adjoint_gradient_pointwise(u, w, s, omega, h), u


def misfit(s, omega, h, source, receivers, d, tol=1e-10):
    b = point_source_rhs(s.shape, h, [source])[0]
    u = solve_forward(s, omega, h, b, tol).x
    return 0.5 * float(np.sum(np.abs(sample(u, receivers) - d) ** 2))
