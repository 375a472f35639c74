"""Discretisation of the Helmholtz problem (oracle; test infrastructure only).

Paper section 2: -Laplace(u) - k(x)^2 u = b on a parallelepiped, Dirichlet
(u = g) or first-order Sommerfeld (du/dn - i k u = 0) boundary conditions.
Section 2.4: vertex-centred grid with equal spacing h, second-order 7-point
stencil, A_h = -Laplace_h - k^2 I (eq. Helmstencil); at Sommerfeld boundary
nodes a ghost point outside the domain is eliminated with
    u_ghost = u_mirror + 2 h i k u_boundary          (eq. elimination).
Section 3.3: the CSLP operator M_h = -Laplace_h - (beta1 - beta2 i) k^2 I;
the paper's default is beta1 = 1, beta2 = -0.5, i.e. M = -Laplace_h - (1 + 0.5i) k^2.
Section 3.4.4: coarse operators are rediscretised with the same boundary
conditions, so the ghost elimination uses the unshifted k in M as in A.

Readings where the paper is silent (all also listed in the design notes):
* Edges and corners: each missing neighbour is eliminated independently
  along its own axis; a node on n_j faces gets n_j diagonal terms -2ik/h.
* Dirichlet: the unknowns are the interior nodes; boundary nodes carry the
  data g.  With g = 0 the boundary entries are stored zeros.

Arrays are C-contiguous (..., nz, ny, nx) with x fastest (the paper's
i1-fastest loop order of Algorithm 2); any leading batch axes are allowed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

DIRICHLET = "dirichlet"
SOMMERFELD = "sommerfeld"


@dataclass
class Level:
    """One grid of the hierarchy.

    shape : (nz, ny, nx) nodes including the boundary
    h     : spacing
    k     : real wavenumber per node (used by the Sommerfeld ghost term)
    bc    : "dirichlet" | "sommerfeld"
    """

    shape: tuple
    h: float
    k: np.ndarray
    bc: str

    @property
    def k2(self):
        return self.k * self.k


def boundary_directions(shape) -> np.ndarray:
    """n_j = number of grid faces node j lies on (0 interior, 1 face, 2 edge, 3 corner)."""
    n = np.zeros(shape, dtype=np.int64)
    for ax, m in enumerate(shape):
        idx = np.arange(m)
        on = ((idx == 0) | (idx == m - 1)).astype(np.int64)
        sh = [1, 1, 1]
        sh[ax] = m
        n = n + on.reshape(sh)
    return n


def unknown_mask(shape, bc) -> np.ndarray:
    """True where a node is an unknown: all nodes (Sommerfeld), interior (Dirichlet)."""
    if bc == SOMMERFELD:
        return np.ones(shape, dtype=bool)
    m = np.zeros(shape, dtype=bool)
    m[1:-1, 1:-1, 1:-1] = True
    return m


def _zero_boundary(x):
    y = x.copy()
    y[..., 0, :, :] = 0
    y[..., -1, :, :] = 0
    y[..., :, 0, :] = 0
    y[..., :, -1, :] = 0
    y[..., :, :, 0] = 0
    y[..., :, :, -1] = 0
    return y


def apply_operator(x, vol, k, h, bc):
    """y = (-Laplace_h - vol) x, matrix-free (Algorithm 2).

    vol : complex or real per-node volume coefficient (k^2 for A_h,
          (beta1 - beta2 i) k^2 for M_h)
    k   : real wavenumber per node, used only in the Sommerfeld ghost points
    The result has the dtype of x (complex64 arithmetic stays complex64).
    """
    x = np.asarray(x)
    cdt = x.dtype
    if bc == DIRICHLET:
        x = _zero_boundary(x)
    pad = [(0, 0)] * (x.ndim - 3) + [(1, 1)] * 3
    xp = np.pad(x, pad)
    if bc == SOMMERFELD:
        # ghost = mirror + 2 h i k * boundary value, on each of the six faces
        two_hik = (2j * h * k).astype(cdt)
        xp[..., 0, 1:-1, 1:-1] = x[..., 1, :, :] + two_hik[0, :, :] * x[..., 0, :, :]
        xp[..., -1, 1:-1, 1:-1] = x[..., -2, :, :] + two_hik[-1, :, :] * x[..., -1, :, :]
        xp[..., 1:-1, 0, 1:-1] = x[..., :, 1, :] + two_hik[:, 0, :] * x[..., :, 0, :]
        xp[..., 1:-1, -1, 1:-1] = x[..., :, -2, :] + two_hik[:, -1, :] * x[..., :, -1, :]
        xp[..., 1:-1, 1:-1, 0] = x[..., :, :, 1] + two_hik[:, :, 0] * x[..., :, :, 0]
        xp[..., 1:-1, 1:-1, -1] = x[..., :, :, -2] + two_hik[:, :, -1] * x[..., :, :, -1]
    c = xp[..., 1:-1, 1:-1, 1:-1]
    # the stencil's 6 x_j - sum x_nb, summed as six differences x_j - x_nb (the
    # same operator; the grouping keeps single-precision evaluations accurate
    # for smooth x)
    lap = ((c - xp[..., :-2, 1:-1, 1:-1]) + (c - xp[..., 2:, 1:-1, 1:-1])
           + (c - xp[..., 1:-1, :-2, 1:-1]) + (c - xp[..., 1:-1, 2:, 1:-1])
           + (c - xp[..., 1:-1, 1:-1, :-2]) + (c - xp[..., 1:-1, 1:-1, 2:]))
    y = lap * (1.0 / (h * h)) - vol.astype(cdt) * c
    if bc == DIRICHLET:
        y = _zero_boundary(y)
    return y.astype(cdt)


def cslp_shift(beta1=1.0, beta2=-0.5):
    """Complex factor (beta1 - beta2 i) multiplying k^2 in M_h (section 3.3)."""
    return complex(beta1, -beta2)


def apply_A(x, lvl: Level):
    """y = A_h x with A_h = -Laplace_h - k^2 I (eq. Helmstencil)."""
    return apply_operator(x, lvl.k2, lvl.k, lvl.h, lvl.bc)


def apply_M(x, lvl: Level, beta1=1.0, beta2=-0.5):
    """y = M_h x with M_h = -Laplace_h - (beta1 - beta2 i) k^2 I (eq. preconditioner)."""
    return apply_operator(x, cslp_shift(beta1, beta2) * lvl.k2, lvl.k, lvl.h, lvl.bc)


def diag_M(lvl: Level, beta1=1.0, beta2=-0.5, dtype=np.complex128):
    """Diagonal of M_h including the ghost-elimination terms -2ik/h per face.

    Dirichlet boundary nodes are not unknowns; their entry is set to 1 so that
    a Jacobi step leaves their (zero) value untouched.
    """
    h = lvl.h
    d = 6.0 / (h * h) - cslp_shift(beta1, beta2) * lvl.k2
    if lvl.bc == SOMMERFELD:
        d = d - boundary_directions(lvl.shape) * (2j * lvl.k / h)
    else:
        d = np.where(unknown_mask(lvl.shape, lvl.bc), d, 1.0)
    return d.astype(dtype)


def point_source_rhs(shape, h, nodes, dtype=np.complex128):
    """Discrete Dirac right-hand sides (section 2.4): 1/h^3 at the source node.

    nodes : list of (iz, iy, ix); returns (len(nodes), nz, ny, nx).
    """
    b = np.zeros((len(nodes),) + tuple(shape), dtype=dtype)
    for r, (iz, iy, ix) in enumerate(nodes):
        b[r, iz, iy, ix] = 1.0 / h**3
    return b


def closed_off_problem(n, k):
    """Closed-off problem of section 2.1 on n^3 nodes of the unit cube.

    b = (21 pi^2 - k^2) sin(pi x) sin(2 pi y) sin(4 pi z) - k^2, u = 1 on the
    boundary, exact solution u* = sin(pi x) sin(2 pi y) sin(4 pi z) + 1.
    The Dirichlet data are lifted into the right-hand side: each interior node
    adjacent to the boundary gets +g/h^2 per boundary neighbour (the boundary
    neighbour's coupling -1/h^2 times the known value g = 1 moved to the
    right-hand side).  Returns (level, b, u_exact) with b and u_exact zero on
    the boundary, i.e. in the unknowns-only form of a homogeneous problem.
    """
    h = 1.0 / (n - 1)
    t = np.linspace(0.0, 1.0, n)
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    sss = np.sin(np.pi * x) * np.sin(2 * np.pi * y) * np.sin(4 * np.pi * z)
    b = (21 * np.pi**2 - k**2) * sss - k**2
    g = 1.0
    lift = np.zeros((n, n, n))
    lift[1, :, :] += g
    lift[-2, :, :] += g
    lift[:, 1, :] += g
    lift[:, -2, :] += g
    lift[:, :, 1] += g
    lift[:, :, -2] += g
    b = b + lift / h**2
    interior = unknown_mask((n, n, n), DIRICHLET)
    b = np.where(interior, b, 0.0).astype(np.complex128)
    u_exact = np.where(interior, sss + 1.0, 0.0)
    lvl = Level((n, n, n), h, np.full((n, n, n), float(k)), DIRICHLET)
    return lvl, b, u_exact
