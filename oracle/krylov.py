"""Right-preconditioned Bi-CGSTAB (oracle; test infrastructure only).

The paper uses Bi-CGSTAB (van der Vorst 1992) with right preconditioning
(section 3.2), so the recursively updated residual is the true one, and stops
when ||b - A u_k||_2 / ||b||_2 <= 1e-6 (section 5, stopping criterion of
Bi-CGSTAB and IDR(s)).  The algorithm text is not printed in the paper; this
is the standard form:

    r = b - A x0, r_hat = r, rho_old = alpha = omega = 1, p = v = 0
    repeat
        rho  = <r_hat, r>                      (Hermitian: conjugate first argument)
        beta = (rho / rho_old) (alpha / omega)
        p    = r + beta (p - omega v)
        p_hat = K p                            (K = one multigrid V-cycle on M)
        v    = A p_hat
        alpha = rho / <r_hat, v>
        s    = r - alpha v
        if ||s|| / ||b|| <= tol: x += alpha p_hat, stop   (half step)
        s_hat = K s
        t    = A s_hat
        omega = <t, s> / <t, t>
        x   += alpha p_hat + omega s_hat
        r    = s - omega t
        stop if ||r|| / ||b|| <= tol
        rho_old = rho

After the loop the true residual b - A x is computed; if it misses the
tolerance (rounding drift between the recursive and the true residual) the
iteration restarts from x.  Breakdown (|rho|, |<r_hat, v>| or |omega| tiny
relative to the scale of the quantities involved) ends with status BREAKDOWN.

Counting: ``iterations`` counts full steps, a half-step exit adds 0.5;
``matvecs`` counts A-products, with the paper's convention of also counting
the initial residual (all printed Bi-CGSTAB counts are odd).
"""
from __future__ import annotations

import enum
from dataclasses import dataclass, field

import numpy as np


class Status(enum.IntEnum):
    OK = 0
    BREAKDOWN = 5
    NOT_CONVERGED = 6


@dataclass
class SolveResult:
    x: np.ndarray
    status: Status
    iterations: float
    matvecs: int
    relres: float            # recursive residual norm / ||b|| at exit
    relres_true: float       # ||b - A x|| / ||b||
    history: list = field(default_factory=list)


def _vdot(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


def _norm(a):
    return float(np.linalg.norm(a.ravel()))


def bicgstab(apply_A, precond, b, x0=None, tol=1e-6, maxit=1000, max_restarts=5,
             breakdown_tol=1e-300, fixed_iterations=None) -> SolveResult:
    """Solve A x = b.  ``apply_A`` and ``precond`` map arrays of b's shape.

    fixed_iterations : run exactly this many full steps with no stopping test
                       (used to compare iterates).
    """
    b = np.asarray(b)
    bnorm = _norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=b.dtype)
    if bnorm == 0.0:
        return SolveResult(np.zeros_like(b), Status.OK, 0, 0, 0.0, 0.0)
    history = []
    iters = 0.0
    matvecs = 1                      # initial residual, paper convention
    restarts = 0
    status = Status.NOT_CONVERGED
    relres = np.inf
    while True:
        r = b - apply_A(x) if (x0 is not None or restarts > 0) else b.copy()
        r_hat = r.copy()
        rho_old = alpha = omega = 1.0 + 0j
        p = np.zeros_like(b)
        v = np.zeros_like(b)
        converged = False
        while iters < maxit or fixed_iterations is not None:
            if fixed_iterations is not None and iters >= fixed_iterations:
                break
            rho = _vdot(r_hat, r)
            if abs(rho) <= breakdown_tol * _norm(r_hat) * _norm(r):
                status = Status.BREAKDOWN
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            p_hat = precond(p)
            v = apply_A(p_hat)
            matvecs += 1
            rv = _vdot(r_hat, v)
            if abs(rv) <= breakdown_tol * _norm(r_hat) * _norm(v):
                status = Status.BREAKDOWN
                break
            alpha = rho / rv
            s = r - alpha * v
            snorm = _norm(s) / bnorm
            if fixed_iterations is None and snorm <= tol:
                x = x + alpha * p_hat
                iters += 0.5
                relres = snorm
                history.append(snorm)
                converged = True
                break
            s_hat = precond(s)
            t = apply_A(s_hat)
            matvecs += 1
            tt = _vdot(t, t)
            if tt == 0.0:
                status = Status.BREAKDOWN
                break
            omega = _vdot(t, s) / tt
            x = x + alpha * p_hat + omega * s_hat
            r = s - omega * t
            iters += 1
            relres = _norm(r) / bnorm
            history.append(relres)
            if fixed_iterations is None and relres <= tol:
                converged = True
                break
            if abs(omega) <= breakdown_tol:
                status = Status.BREAKDOWN
                break
            rho_old = rho
        if fixed_iterations is not None:
            status = Status.OK
            break
        if status == Status.BREAKDOWN:
            break
        if not converged:
            status = Status.NOT_CONVERGED
            break
        true_rel = _norm(b - apply_A(x)) / bnorm
        if true_rel <= tol:
            status = Status.OK
            break
        restarts += 1
        if restarts > max_restarts or iters >= maxit:
            status = Status.NOT_CONVERGED
            break
        matvecs += 1
    true_rel = _norm(b - apply_A(x)) / bnorm
    return SolveResult(x, status, iters, matvecs, relres, true_rel, history)
