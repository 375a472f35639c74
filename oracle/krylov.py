"""Right-preconditioned Bi-CGSTAB and IDR(s), left-preconditioned full GMRES
(oracle; test infrastructure only).

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
             breakdown_tol=1e-300, fixed_iterations=None, shadow_dtype=None,
             restart_decade=False) -> SolveResult:
    """Solve A x = b.  ``apply_A`` and ``precond`` map arrays of b's shape.

    fixed_iterations : run exactly this many full steps with no stopping test
                       (used to compare iterates).
    shadow_dtype     : None keeps r_hat = r (the standard choice); a dtype
                       such as complex64 takes r_hat = r rounded to it (then
                       widened back), the shadow vector of a solve whose
                       preconditioner runs in that precision.  Bi-CGSTAB
                       admits any fixed r_hat with <r_hat, r> != 0.
    restart_decade   : restart from the current x (true residual, new shadow
                       residual, fresh recurrences) each time ||r|| / ||b||
                       falls below the next power of ten (0.1, 0.01, ...),
                       also with fixed_iterations; each restart counts one
                       product with A.  Not part of the paper's method: the
                       policy of the mixed form, whose rounded preconditioner
                       is not exactly linear.
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
    decades = 0
    status = Status.NOT_CONVERGED
    relres = np.inf
    next_decade = 0.1
    if restart_decade and x0 is not None:
        r0 = _norm(b - apply_A(x)) / bnorm
        while next_decade >= r0:
            next_decade *= 0.1
    while True:
        r = b - apply_A(x) if (x0 is not None or restarts > 0 or decades > 0) else b.copy()
        r_hat = r.copy() if shadow_dtype is None else r.astype(shadow_dtype).astype(r.dtype)
        rho_old = alpha = omega = 1.0 + 0j
        p = np.zeros_like(b)
        v = np.zeros_like(b)
        converged = False
        decade = False
        if decades > 0 and _norm(r) / bnorm <= tol and fixed_iterations is None:
            # the true residual at a restart already meets the tolerance
            relres = _norm(r) / bnorm
            status = Status.OK
            break
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
            limit = fixed_iterations if fixed_iterations is not None else maxit
            if restart_decade and relres <= next_decade and iters < limit:
                while next_decade >= relres:
                    next_decade *= 0.1
                decade = True
                break
            rho_old = rho
        if decade:
            decades += 1
            matvecs += 1
            continue
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


def idrs(apply_A, precond, b, P, x0=None, tol=1e-6, maxit=2000, kappa=0.7, max_restarts=5,
         breakdown_tol=1e-300, fixed_steps=None, monitor=None) -> SolveResult:
    """Solve A x = b by right-preconditioned IDR(s), s = len(P) (section 3.1:
    the paper's IDR(4), after Sonneveld and van Gijzen; stopped, like
    Bi-CGSTAB, on the true relative residual of section 5).

    The paper does not print the algorithm.  This is the biorthogonal variant
    (van Gijzen and Sonneveld, ACM TOMS 38(1), 2011), with the preconditioner
    K (one multigrid cycle on M) applied on the right so that r stays the
    residual b - A x of the unpreconditioned system:

        r = b - A x;  G = U = 0 (s vectors each);  Ms = I (s x s);  om = 1
        repeat
            f = P^H r                                   (f_i = <p_i, r>)
            for k = 1 .. s
                c = Ms[k:s, k:s]^-1 f[k:s]              (lower triangular)
                v = K (r - sum_{j>=k} c_j g_j)
                u_k = sum_{j>=k} c_j u_j + om v
                g_k = A u_k
                for i = 1 .. k-1                         (make g_k orthogonal to p_1..p_{k-1})
                    a = <p_i, g_k> / Ms[i, i]
                    g_k -= a g_i;  u_k -= a u_i
                Ms[i, k] = <p_i, g_k>  for i = k .. s
                beta = f_k / Ms[k, k]
                r -= beta g_k;  x += beta u_k           (now r is orthogonal to p_1..p_k)
                stop if ||r|| / ||b|| <= tol
                f[k+1:s] -= beta Ms[k+1:s, k]
            v = K r;  t = A v                            (dimension reduction)
            om = <t, r> / <t, t>,  enlarged by kappa / rho when
                 rho = |<t, r>| / (||t|| ||r||) < kappa   (kappa = 0.7; 0 disables)
            x += om v;  r -= om t
            stop if ||r|| / ||b|| <= tol

    Counting: ``iterations`` = products with A after the initial residual
    (s + 1 per cycle); ``matvecs`` adds the initial residual (and one per
    restart), the paper's #Matvec.  After the loop the true residual decides,
    as in ``bicgstab``: a miss restarts from x with G = U = 0.

    P           : array (s,) + b.shape of shadow vectors (linearly independent).
    fixed_steps : stop after exactly this many A-products, no stopping test.
    monitor     : optional callable(k, x, r, G, U, Ms) after every update of r
                  (k = inner step 0 .. s-1, or s for the reduction step).
    """
    b = np.asarray(b)
    P = np.asarray(P)
    s_dim = P.shape[0]
    bnorm = _norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=b.dtype)
    if bnorm == 0.0:
        return SolveResult(np.zeros_like(b), Status.OK, 0, 0, 0.0, 0.0)
    history = []
    steps = 0
    matvecs = 1
    restarts = 0
    status = Status.NOT_CONVERGED
    relres = np.inf

    def done():
        if fixed_steps is not None:
            return steps >= fixed_steps
        return relres <= tol

    while True:
        r = b - apply_A(x) if (x0 is not None or restarts > 0) else b.copy()
        relres = _norm(r) / bnorm
        G = np.zeros((s_dim,) + b.shape, dtype=b.dtype)
        U = np.zeros((s_dim,) + b.shape, dtype=b.dtype)
        Ms = np.eye(s_dim, dtype=np.complex128)
        om = 1.0 + 0j
        stop = done()
        while not stop and (steps < maxit or fixed_steps is not None):
            f = np.array([_vdot(P[i], r) for i in range(s_dim)])
            for k in range(s_dim):
                c = np.linalg.solve(np.tril(Ms[k:, k:]), f[k:])
                v = r.copy()
                for j in range(k, s_dim):
                    v = v - c[j - k] * G[j]
                v = precond(v)
                uk = om * v
                for j in range(k, s_dim):
                    uk = uk + c[j - k] * U[j]
                U[k] = uk
                G[k] = apply_A(U[k])
                steps += 1
                matvecs += 1
                for i in range(k):
                    a = _vdot(P[i], G[k]) / Ms[i, i]
                    G[k] = G[k] - a * G[i]
                    U[k] = U[k] - a * U[i]
                for i in range(k, s_dim):
                    Ms[i, k] = _vdot(P[i], G[k])
                if abs(Ms[k, k]) <= breakdown_tol * _norm(P[k]) * _norm(G[k]):
                    status = Status.BREAKDOWN
                    stop = True
                    break
                beta = f[k] / Ms[k, k]
                r = r - beta * G[k]
                x = x + beta * U[k]
                relres = _norm(r) / bnorm
                history.append(relres)
                if monitor is not None:
                    monitor(k, x, r, G, U, Ms)
                if done() or (fixed_steps is None and steps >= maxit):
                    stop = True
                    break
                f[k + 1:] = f[k + 1:] - beta * Ms[k + 1:, k]
            if stop:
                break
            v = precond(r)
            t = apply_A(v)
            steps += 1
            matvecs += 1
            tt = _vdot(t, t)
            if tt == 0.0:
                status = Status.BREAKDOWN
                break
            tr = _vdot(t, r)
            om = tr / tt
            rho = abs(tr) / (np.sqrt(tt.real) * _norm(r))
            if rho < kappa:
                om = om * kappa / rho
            if abs(om) <= breakdown_tol:
                status = Status.BREAKDOWN
                break
            x = x + om * v
            r = r - om * t
            relres = _norm(r) / bnorm
            history.append(relres)
            if monitor is not None:
                monitor(s_dim, x, r, G, U, Ms)
            stop = done()
        if fixed_steps is not None:
            status = Status.OK
            break
        if status == Status.BREAKDOWN:
            break
        if relres > tol:
            status = Status.NOT_CONVERGED
            break
        true_rel = _norm(b - apply_A(x)) / bnorm
        if true_rel <= tol:
            status = Status.OK
            break
        restarts += 1
        if restarts > max_restarts or steps >= maxit:
            status = Status.NOT_CONVERGED
            break
        matvecs += 1
    true_rel = _norm(b - apply_A(x)) / bnorm
    return SolveResult(x, status, steps, matvecs, relres, true_rel, history)


def gmres(apply_A, precond, b, x0=None, tol=1e-6, maxit=1000, monitor=None) -> SolveResult:
    """Solve A x = b by full GMRES on the left-preconditioned system
    K A x = K b, K = one multigrid cycle on M (sections 3.1, 3.2), stopped at
    ||K b - K A x|| / ||K b|| <= tol (the paper's GMRES criterion, section 5).

    No restart.  Arnoldi with modified Gram-Schmidt, Givens rotations for the
    least-squares problem (Saad and Schultz 1986):

        r = K (b - A x0);  beta = ||r||;  v_1 = r / beta;  g = beta e_1
        for j = 1, 2, ...
            w = K A v_j
            for i = 1 .. j:  h_ij = <v_i, w>;  w -= h_ij v_i
            h_{j+1,j} = ||w||;  v_{j+1} = w / h_{j+1,j}
            apply the earlier rotations to column j, then the rotation that
            zeroes h_{j+1,j}; |g_{j+1}| is the preconditioned residual norm
            stop if |g_{j+1}| / ||K b|| <= tol
        x = x0 + V y,  H y = g (upper triangular)

    Counting: ``iterations`` = Arnoldi steps (products with A after the initial
    residual); ``matvecs`` adds the initial residual when x0 is given (with
    x0 = 0 the initial residual is b and costs no product).  ``relres`` is the
    preconditioned relative residual, ``relres_true`` the unpreconditioned one.
    monitor: optional callable(j, V, Hbar) after Arnoldi step j: V the j + 2
    basis vectors, Hbar the (j + 2) x (j + 1) Hessenberg matrix before rotations.
    """
    b = np.asarray(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=b.dtype)
    if _norm(b) == 0.0:
        return SolveResult(np.zeros_like(b), Status.OK, 0, 0, 0.0, 0.0)
    kb = precond(b)
    kbn = _norm(kb)
    matvecs = 0
    if x0 is None:
        r = kb
    else:
        r = precond(b - apply_A(x))
        matvecs += 1
    beta = _norm(r)
    history = [beta / kbn]
    if beta / kbn <= tol:
        true_rel = _norm(b - apply_A(x)) / _norm(b)
        return SolveResult(x, Status.OK, 0, matvecs, beta / kbn, true_rel, history)
    V = [r / beta]
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    Hbar = np.zeros((maxit + 1, maxit), dtype=np.complex128) if monitor is not None else None
    cs = np.zeros(maxit, dtype=np.complex128)
    sn = np.zeros(maxit, dtype=np.complex128)
    g = np.zeros(maxit + 1, dtype=np.complex128)
    g[0] = beta
    status = Status.NOT_CONVERGED
    m = 0
    relres = beta / kbn
    for j in range(maxit):
        w = precond(apply_A(V[j]))
        matvecs += 1
        for i in range(j + 1):
            H[i, j] = _vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = _norm(w)
        if monitor is not None and H[j + 1, j] != 0.0:
            Hbar[: j + 2, j] = H[: j + 2, j]
            monitor(j, V + [w / H[j + 1, j]], Hbar[: j + 2, : j + 1])
        # earlier rotations on the new column
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
            H[i, j] = t
        # rotation zeroing H[j+1, j]:  [c s; -conj(s) conj(c)] with c real
        a, bb = H[j, j], H[j + 1, j]
        den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
        if den == 0.0:
            status = Status.BREAKDOWN
            m = j
            break
        cs[j] = abs(a) / den
        sn[j] = (a / abs(a)) * np.conj(bb) / den if a != 0 else 1.0
        H[j, j] = cs[j] * a + sn[j] * bb
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        m = j + 1
        relres = abs(g[j + 1]) / kbn
        history.append(relres)
        if relres <= tol:
            status = Status.OK
            break
        if H[j + 1, j] == 0.0 and den == 0.0:
            break
        V.append(w / _norm(w))
    y = np.zeros(m, dtype=np.complex128)
    for i in range(m - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1: m] @ y[i + 1: m]) / H[i, i]
    for i in range(m):
        x = x + y[i] * V[i]
    true_rel = _norm(b - apply_A(x)) / _norm(b)
    return SolveResult(x, status, m, matvecs, relres, true_rel, history)
