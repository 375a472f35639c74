"""Geometric multigrid for the CSLP preconditioner (oracle; test infrastructure only).

Paper section 3.4 and Algorithm 1 (two-grid cycle), applied recursively as
a V-cycle, or an F-cycle, with one pre- and one post-smoothing step per level
(section 3.4.5):

* smoother: damped Jacobi with omega = 0.8 (section 3.4.1),
      u <- u + omega D^{-1} (b - M u),  D = diag(M) incl. boundary terms;
* restriction: 3D full weighting, stencil 1/64 [1 2 1] x [1 2 1] x [1 2 1]
  evaluated at the even fine nodes (eq. matrix-free restriction);
* prolongation: trilinear interpolation, the eight cases of eq.
  matrix-free prolongation (copy, 2-, 4- and 8-point averages);
* coarse operators: rediscretisation (DCG, section 3.4.4) on H = 2h with the
  same boundary conditions;
* coarse node i <-> fine node 2i (0-based form of the 1-based map
  i_c <-> 2 i_c - 1 of section 4.2).

Readings where the paper is silent (also in the design notes):
* wavenumber on coarse grids: injection k_{l+1}(i) = k_l(2i);
* restriction at Sommerfeld boundary nodes: the missing fine node outside the
  domain takes the value of its mirror image (even reflection), so constants
  are preserved; Dirichlet coarse boundary nodes are not unknowns (zero);
* zero initial guess on every level, so one V-cycle is a fixed linear map;
* coarsest level: solved exactly (sparse LU of the rediscretised M) by
  default, or, as the paper does (end of section 3.4.5, section 4.2 and the
  coarse stopping criterion of section 5), by full GMRES without
  preconditioning from a zero initial guess to relative residual 1e-11
  (``coarse="gmres"``), always in complex128; the two agree to about 1e-11;
* level count: coarsen while the next level keeps at least 3 nodes per axis,
  or a given count, or (``paper17``) while every axis has more than 17 nodes,
  which reproduces the paper's 17^3 and 41 x 41 x 13 coarsest grids.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from .discretization import (
    DIRICHLET,
    SOMMERFELD,
    Level,
    apply_M,
    diag_M,
    unknown_mask,
)
from .krylov import gmres


def coarsen_shape(shape):
    return tuple((m - 1) // 2 + 1 for m in shape)


def level_shapes(shape, n_levels=0, rule="min3"):
    """List of per-level shapes, finest first."""
    for m in shape:
        if m < 3 or m % 2 == 0:
            raise ValueError("every axis needs an odd node count >= 3")
    shapes = [tuple(shape)]
    if n_levels and n_levels > 0:
        for _ in range(n_levels - 1):
            s = shapes[-1]
            if any((m - 1) % 2 for m in s) or min(s) < 5:
                raise ValueError(f"cannot coarsen {s} to {n_levels} levels")
            shapes.append(coarsen_shape(s))
        return shapes
    while True:
        s = shapes[-1]
        if any((m - 1) % 2 for m in s):
            break
        if rule == "paper17":
            if not all(m > 17 for m in s):
                break
        elif min(coarsen_shape(s)) < 3:
            break
        shapes.append(coarsen_shape(s))
    return shapes


@dataclass
class Hierarchy:
    """Grids of the V-cycle plus the factorised coarsest operator."""

    levels: list
    beta1: float = 1.0
    beta2: float = -0.5
    omega: float = 0.8
    dtype: type = np.complex128
    coarse_lu: object = None
    coarse_mask: np.ndarray = None
    diags: list = field(default_factory=list)
    coarse: str = "exact"          # coarsest solve: "exact" (sparse LU) or "gmres"
    coarse_tol: float = 1e-11      # relative residual of the coarsest GMRES
    coarse_maxit: int = 200        # Arnoldi steps of the coarsest GMRES (no restart)
    coarse_level64: Level = None   # the coarsest level in double precision (for GMRES)

    @property
    def coarsest(self):
        return self.levels[-1]


def _level_in_precision(lvl: Level, dtype):
    if dtype == np.complex64:
        return Level(lvl.shape, lvl.h, lvl.k.astype(np.float32), lvl.bc)
    return lvl


def build_hierarchy(k, h, bc, n_levels=0, rule="min3", beta1=1.0, beta2=-0.5,
                    omega=0.8, dtype=np.complex128, coarse="exact", coarse_tol=1e-11,
                    coarse_maxit=200) -> Hierarchy:
    """Levels by injection of k, then a sparse LU of the coarsest M.

    dtype complex64 gives the mixed-precision variant: k^2, M, D and the
    coarse factorisation in single precision.  coarse="gmres" solves the
    coarsest level by full GMRES in complex128 instead (see coarse_gmres).
    """
    if coarse not in ("exact", "gmres"):
        raise ValueError("coarse must be 'exact' or 'gmres'")
    shapes = level_shapes(k.shape, n_levels, rule)
    levels = [Level(shapes[0], h, np.asarray(k, dtype=np.float64), bc)]
    for s in shapes[1:]:
        prev = levels[-1]
        levels.append(Level(s, prev.h * 2.0, prev.k[::2, ::2, ::2].copy(), bc))
    coarsest64 = levels[-1]
    levels = [_level_in_precision(lv, dtype) for lv in levels]
    hier = Hierarchy(levels, beta1, beta2, omega, dtype, coarse=coarse, coarse_tol=coarse_tol,
                     coarse_maxit=coarse_maxit, coarse_level64=coarsest64)
    hier.diags = [diag_M(lv, beta1, beta2, dtype) for lv in levels]
    hier.coarse_mask = unknown_mask(hier.coarsest.shape, bc)
    hier.coarse_lu = _factor_coarsest(hier)
    return hier


def _assemble_coarsest(hier: Hierarchy):
    """Sparse matrix of the coarsest M (unknowns only), column by column
    from the matrix-free apply of unit vectors."""
    lvl = hier.coarsest
    mask = hier.coarse_mask
    idx = np.flatnonzero(mask.ravel())
    n = idx.size
    cols, rows, vals = [], [], []
    batch = 256
    for c0 in range(0, n, batch):
        cs = idx[c0:c0 + batch]
        e = np.zeros((cs.size,) + lvl.shape, dtype=hier.dtype)
        e.reshape(cs.size, -1)[np.arange(cs.size), cs] = 1
        y = apply_M(e, lvl, hier.beta1, hier.beta2).reshape(cs.size, -1)[:, idx]
        for j in range(cs.size):
            nz = np.flatnonzero(y[j])
            rows.append(nz)
            cols.append(np.full(nz.size, c0 + j))
            vals.append(y[j, nz])
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n), dtype=hier.dtype)


def _factor_coarsest(hier: Hierarchy):
    return splu(_assemble_coarsest(hier))


def coarse_gmres(b, hier: Hierarchy):
    """The paper's coarsest-grid solve: full GMRES on M_c (no preconditioner,
    no restart), zero initial guess, stopped when the relative residual
    ||b - M_c e|| / ||b|| (the Arnoldi estimate |g_{j+1}| / ||b||) reaches
    hier.coarse_tol, or after hier.coarse_maxit steps.  Always complex128 (the
    operator from the double-precision k of the coarsest level); one
    right-hand side (nz, ny, nx).  Returns (e, Arnoldi steps)."""
    lvl = hier.coarse_level64
    mask = hier.coarse_mask
    b64 = np.asarray(b, dtype=np.complex128) * mask

    def apply(x):
        return apply_M(x * mask, lvl, hier.beta1, hier.beta2) * mask

    res = gmres(apply, lambda v: v, b64, tol=hier.coarse_tol, maxit=hier.coarse_maxit)
    return res.x * mask, res.iterations


def coarse_solve(b, hier: Hierarchy):
    """e = M_c^{-1} b on the coarsest level (unknown nodes only): exactly, or
    by coarse_gmres when the hierarchy was built with coarse="gmres"."""
    if hier.coarse == "gmres":
        if b.ndim == 3:
            return coarse_gmres(b, hier)[0].astype(hier.dtype)
        return np.stack([coarse_gmres(b[r], hier)[0] for r in range(b.shape[0])]).astype(hier.dtype)
    mask = hier.coarse_mask
    e = np.zeros_like(b)
    flat_b = b.reshape(b.shape[:-3] + (-1,))
    flat_e = e.reshape(e.shape[:-3] + (-1,))
    sel = mask.ravel()
    if flat_b.ndim == 1:
        flat_e[sel] = hier.coarse_lu.solve(flat_b[sel])
    else:
        for r in range(flat_b.shape[0]):
            flat_e[r, sel] = hier.coarse_lu.solve(flat_b[r, sel])
    return e


def jacobi_sweep(u, b, lvl: Level, dinv_omega, beta1=1.0, beta2=-0.5):
    """One damped-Jacobi step u + omega D^{-1} (b - M u) (section 3.4.1)."""
    return u + dinv_omega * (b - apply_M(u, lvl, beta1, beta2))


def restrict_fw(r, bc):
    """b_H = I_h^H r_h: full weighting at coarse node I = fine node 2I.

    Written as the 27-term weighted sum of eq. matrix-free restriction: weight
    8 at the centre, 4 for the 6 face neighbours, 2 for the 12 edge
    neighbours, 1 for the 8 corners, all over 64.  Fine nodes outside the
    domain (only reached from Sommerfeld boundary coarse nodes) take the value
    of their mirror image.
    """
    pad = [(0, 0)] * (r.ndim - 3) + [(1, 1)] * 3
    rp = np.pad(r, pad, mode="reflect")
    fine = r.shape[-3:]
    coarse = coarsen_shape(fine)
    out = np.zeros(r.shape[:-3] + coarse, dtype=r.dtype)
    weight = {-1: 1, 0: 2, 1: 1}
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                w = weight[dz] * weight[dy] * weight[dx]
                sl = rp[..., 1 + dz: 1 + dz + fine[0]: 2,
                        1 + dy: 1 + dy + fine[1]: 2,
                        1 + dx: 1 + dx + fine[2]: 2]
                out = out + (w / 64.0) * sl
    return out.astype(r.dtype)


def prolong_trilinear(e, fine_shape):
    """e_h = I_H^h e_H: the eight cases of eq. matrix-free prolongation.

    Fine node (2I + a) with a in {0, 1}^3 averages the coarse nodes
    I + {0, a_z} x {0, a_y} x {0, a_x} (1, 2, 4 or 8 of them).
    """
    out = np.zeros(e.shape[:-3] + tuple(fine_shape), dtype=e.dtype)
    for az in (0, 1):
        for ay in (0, 1):
            for ax in (0, 1):
                acc = 0
                cnt = 0
                for cz in range(az + 1):
                    for cy in range(ay + 1):
                        for cx in range(ax + 1):
                            nz = e.shape[-3] - az
                            ny = e.shape[-2] - ay
                            nx = e.shape[-1] - ax
                            acc = acc + e[..., cz:cz + nz, cy:cy + ny, cx:cx + nx]
                            cnt += 1
                out[..., az::2, ay::2, ax::2] = acc * (1.0 / cnt)
    return out


def vcycle(b, hier: Hierarchy, level=0):
    """u ~= M_l^{-1} b by one V(1,1) cycle with zero initial guess (Algorithm 1
    applied recursively; the coarsest level is solved exactly)."""
    lvl = hier.levels[level]
    if level == len(hier.levels) - 1:
        return coarse_solve(b, hier)
    wd = (hier.omega / hier.diags[level]).astype(hier.dtype)
    u = np.zeros_like(b)
    u = jacobi_sweep(u, b, lvl, wd, hier.beta1, hier.beta2)          # pre-smoothing
    r = b - apply_M(u, lvl, hier.beta1, hier.beta2)                  # residual
    bc_ = restrict_fw(r, lvl.bc)                                     # restriction
    if lvl.bc == DIRICHLET:
        bc_ = bc_ * unknown_mask(hier.levels[level + 1].shape, DIRICHLET)
    e = vcycle(bc_, hier, level + 1)                                 # coarse error
    u = u + prolong_trilinear(e, lvl.shape)                          # correction
    u = jacobi_sweep(u, b, lvl, wd, hier.beta1, hier.beta2)          # post-smoothing
    if lvl.bc == DIRICHLET:
        u = u * unknown_mask(lvl.shape, DIRICHLET)
    return u.astype(hier.dtype)


def fcycle(b, hier: Hierarchy, level=0):
    """u ~= M_l^{-1} b by one F(1,1) cycle with zero initial guess (section
    3.4.5).  The cycle first descends to the coarsest grid; on the way back up,
    every level reached for the first time gets one more V-cycle down to the
    coarsest grid.  Written recursively: as the V-cycle, but the coarse error
    equation is solved by one F-cycle followed by one V-cycle on the coarse
    residual that F-cycle leaves.  On the coarsest level the F-cycle is the
    exact solve, which leaves no residual, so no further cycle follows there."""
    lvl = hier.levels[level]
    if level == len(hier.levels) - 1:
        return coarse_solve(b, hier)
    wd = (hier.omega / hier.diags[level]).astype(hier.dtype)
    u = np.zeros_like(b)
    u = jacobi_sweep(u, b, lvl, wd, hier.beta1, hier.beta2)          # pre-smoothing
    r = b - apply_M(u, lvl, hier.beta1, hier.beta2)                  # residual
    bc_ = restrict_fw(r, lvl.bc)                                     # restriction
    coarse = hier.levels[level + 1]
    if lvl.bc == DIRICHLET:
        bc_ = bc_ * unknown_mask(coarse.shape, DIRICHLET)
    e = fcycle(bc_, hier, level + 1)                                 # F-cycle on the coarse level
    if level + 1 < len(hier.levels) - 1:
        rc = bc_ - apply_M(e, coarse, hier.beta1, hier.beta2)        # its remaining residual
        e = e + vcycle(rc, hier, level + 1)                          # the additional V-cycle
    u = u + prolong_trilinear(e, lvl.shape)                          # correction
    u = jacobi_sweep(u, b, lvl, wd, hier.beta1, hier.beta2)          # post-smoothing
    if lvl.bc == DIRICHLET:
        u = u * unknown_mask(lvl.shape, DIRICHLET)
    return u.astype(hier.dtype)


def vcycle_mixed_entry(b, hier32: Hierarchy):
    """Mixed-precision preconditioner: complex128 in, complex64 V-cycle, complex128 out."""
    return vcycle(b.astype(np.complex64), hier32).astype(np.complex128)


__all__ = [
    "Hierarchy", "build_hierarchy", "level_shapes", "coarsen_shape", "coarse_solve", "coarse_gmres",
    "jacobi_sweep", "restrict_fw", "prolong_trilinear", "vcycle", "fcycle", "vcycle_mixed_entry",
    "SOMMERFELD", "DIRICHLET",
]
