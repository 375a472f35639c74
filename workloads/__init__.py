"""Seeded synthetic inputs for the Helmholtz solver and its oracle.

This module only builds input data: grids, velocity / wavenumber models,
source and receiver node lists, random vectors and perturbation directions.
It holds none of the solver's arithmetic (no stencil, no transfer operator,
no Krylov step), so both the oracle and the GPU path may draw their inputs
from it.

Models (paper section 2 and the workload definitions below):

* ``constant``  - unit cube with a constant wavenumber (closed-off problem of
  section 2.1 and the large constant-k cube).
* ``wedge``     - three-layer wedge of section 2.2 on a uniform grid of
  129 x 129 x 257 nodes, h = 600/128 m.  The paper's velocity figure is not
  available; the two tilted interfaces are the planes depth = 0.4 L + 0.2 x
  and depth = 0.8 L - 0.2 x in coordinates normalised to the box, velocities
  2000 / 1500 / 3000 m/s from top to bottom.
* ``smoothed_noise`` - Gaussian-smoothed random velocity in [1500, 3000] m/s
  on a 65^3 unit cube (adjoint-gradient workload).

Array layout everywhere: C-contiguous ``(nz, ny, nx)``, x fastest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Workload",
    "constant_cube",
    "wedge_velocity",
    "wedge",
    "big_cube",
    "batched_wedge_sources",
    "smoothed_noise_velocity",
    "adjoint_workload",
    "random_complex",
    "receivers_top_grid",
    "closed_off_rhs",
]


@dataclass
class Workload:
    """A synthetic problem instance.

    k        : real wavenumber per node, float64 (nz, ny, nx)
    h        : grid spacing (equal in all directions)
    bc       : "dirichlet" or "sommerfeld"
    sources  : list of (iz, iy, ix) source nodes (Dirac right-hand sides)
    n_levels : multigrid levels (0 = default coarsening)
    name     : human-readable description with sizes
    """

    k: np.ndarray
    h: float
    bc: str
    sources: list
    n_levels: int
    name: str

    @property
    def shape(self):
        return self.k.shape


def constant_cube(n: int, k: float, bc: str, n_levels: int = 0, source=None) -> Workload:
    """Unit cube with n nodes per axis (h = 1/(n-1)), constant wavenumber k."""
    h = 1.0 / (n - 1)
    kk = np.full((n, n, n), float(k), dtype=np.float64)
    c = (n - 1) // 2
    src = [tuple(source) if source is not None else (c, c, c)]
    return Workload(kk, h, bc, src, n_levels, f"cube{n}^3 k={k:g} {bc}")


def wedge_velocity(nx: int = 129, ny: int = 129, nz: int = 257) -> np.ndarray:
    """Three-layer wedge velocity (m/s), array (nz, ny, nx); iz = 0 is the top face.

    With xi = ix/(nx-1) and zeta = iz/(nz-1) (depth from the top face):
    layer 1 (2000 m/s) above zeta = 0.4 + 0.2 xi, layer 3 (3000 m/s) below
    zeta = 0.8 - 0.2 xi, layer 2 (1500 m/s) in between.  The tests are done in
    integers (5 iz (nx-1) vs ...) so that nodes exactly on a plane go to the
    deeper layer without rounding.  No y dependence.
    """
    ix = np.arange(nx)[None, None, :]
    iz = np.arange(nz)[:, None, None]
    mx, mz = nx - 1, nz - 1
    # zeta < 0.4 + 0.2 xi  <=>  5 iz mx < 2 mz mx + mz ix
    upper = 5 * iz * mx < 2 * mz * mx + mz * ix
    # zeta >= 0.8 - 0.2 xi <=>  5 iz mx >= 4 mz mx - mz ix
    lower = 5 * iz * mx >= 4 * mz * mx - mz * ix
    c = np.where(upper, 2000.0, np.where(lower, 3000.0, 1500.0))
    return np.broadcast_to(c, (nz, ny, nx)).astype(np.float64).copy()


def wedge(freq: float = 10.0, nx: int = 129, ny: int = 129, nz: int = 257,
          n_levels: int = 0) -> Workload:
    """Wedge model (600 x 600 m footprint, uniform h = 600/(nx-1)), Sommerfeld,
    point source at the centre of the top face, k = 2 pi f / c."""
    h = 600.0 / (nx - 1)
    c = wedge_velocity(nx, ny, nz)
    k = 2.0 * math.pi * freq / c
    src = [(0, (ny - 1) // 2, (nx - 1) // 2)]
    return Workload(k, h, "sommerfeld", src, n_levels,
                    f"wedge {nx}x{ny}x{nz} f={freq:g}Hz h={h:g}m")


def closed_off_rhs(n: int, k: float):
    """Data of the closed-off problem of section 2.1 on n^3 nodes of the unit
    cube with constant k: f = (21 pi^2 - k^2) sin(pi x) sin(2 pi y) sin(4 pi z)
    - k^2 in the interior, u = 1 on the boundary.  The boundary value is moved
    into the right-hand side of the interior nodes next to the boundary (g / h^2
    per boundary neighbour, g = 1), so b and the returned exact solution are zero
    on the boundary.  Returns (k array, b complex128, u_exact), all (n, n, n)."""
    h = 1.0 / (n - 1)
    t = np.linspace(0.0, 1.0, n)
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    sss = np.sin(np.pi * x) * np.sin(2 * np.pi * y) * np.sin(4 * np.pi * z)
    f = (21 * np.pi**2 - k**2) * sss - k**2
    near = np.zeros((n, n, n))
    for ax in range(3):
        for i in (1, n - 2):
            idx = [slice(None)] * 3
            idx[ax] = i
            near[tuple(idx)] += 1.0
    interior = np.zeros((n, n, n), dtype=bool)
    interior[1:-1, 1:-1, 1:-1] = True
    b = np.where(interior, f + near / h**2, 0.0).astype(np.complex128)
    u = np.where(interior, sss + 1.0, 0.0)
    return np.full((n, n, n), float(k)), b, u


def big_cube(n: int = 513, k: float = 160.0, n_levels: int = 8) -> Workload:
    """Constant-k Sommerfeld unit cube (513^3, k = 160, kh = 0.3125, 8 levels)."""
    return constant_cube(n, k, "sommerfeld", n_levels=n_levels)


def batched_wedge_sources(nsrc: int = 16, seed: int = 4, nx: int = 129, ny: int = 129,
                          width: float = 600.0) -> list:
    """nsrc distinct source nodes on the top face, (x, y) uniform in the footprint.

    Draws (x, y) ~ U(0, width)^2 from ``default_rng(seed)``, snaps to the
    nearest node, clips to the grid and redraws duplicates.
    """
    rng = np.random.default_rng(seed)
    h = width / (nx - 1)
    out, seen = [], set()
    while len(out) < nsrc:
        xy = rng.uniform(0.0, width, size=2)
        ix = int(np.clip(np.rint(xy[0] / h), 0, nx - 1))
        iy = int(np.clip(np.rint(xy[1] / h), 0, ny - 1))
        if (iy, ix) in seen:
            continue
        seen.add((iy, ix))
        out.append((0, iy, ix))
    return out


def _smooth_minmax(field: np.ndarray, sigma: float, lo: float, hi: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter

    g = gaussian_filter(field, sigma=sigma, mode="reflect", truncate=4.0)
    g = (g - g.min()) / (g.max() - g.min())
    return lo + (hi - lo) * g


def smoothed_noise_velocity(n: int = 65, seed: int = 5, sigma: float = 4.0,
                            cmin: float = 1500.0, cmax: float = 3000.0) -> np.ndarray:
    """Seeded Gaussian noise, smoothed (sigma in cells), mapped to [cmin, cmax]."""
    rng = np.random.default_rng(seed)
    return _smooth_minmax(rng.standard_normal((n, n, n)), sigma, cmin, cmax)


def receivers_top_grid(n: int = 65, m: int = 8, first: int = 4, step: int = 8) -> list:
    """m x m receiver nodes (0, first + step*b, first + step*a) on the top face."""
    return [(0, first + step * b, first + step * a) for b in range(m) for a in range(m)]


@dataclass
class AdjointWorkload:
    """Inputs of the misfit-gradient problem.

    s_model : squared slowness 1/c^2 of the model where the gradient is taken
    s_true  : squared slowness of the perturbed model that generates the data
    omega   : angular frequency (rad/s); k = omega sqrt(s)
    h       : spacing; source: (iz, iy, ix); receivers: list of nodes
    directions : (ndir, n, n, n) float64 perturbation directions, max |v| = 1
    eps     : central finite-difference step on s
    """

    s_model: np.ndarray
    s_true: np.ndarray
    omega: float
    h: float
    source: tuple
    receivers: list
    directions: np.ndarray
    eps: float


def adjoint_workload(n: int = 65, ndir: int = 20) -> AdjointWorkload:
    """65^3 unit cube, smoothed-noise velocity in [1500, 3000] m/s, omega chosen
    so that max kh = 0.5, centre-top source, 8 x 8 receivers on the top face,
    data from a model perturbed by 5 % smoothed noise, ``ndir`` smoothed random
    finite-difference directions."""
    h = 1.0 / (n - 1)
    c = smoothed_noise_velocity(n, seed=5)
    omega = 0.5 * 1500.0 / h
    rng6 = np.random.default_rng(6)
    delta = _smooth_minmax(rng6.standard_normal((n, n, n)), 4.0, -1.0, 1.0)
    c_true = c * (1.0 + 0.05 * delta)
    rng7 = np.random.default_rng(7)
    from scipy.ndimage import gaussian_filter

    dirs = np.empty((ndir, n, n, n))
    for i in range(ndir):
        v = gaussian_filter(rng7.standard_normal((n, n, n)), sigma=2.0, mode="reflect",
                            truncate=4.0)
        dirs[i] = v / np.abs(v).max()
    s = 1.0 / c**2
    c0 = (n - 1) // 2
    recv = receivers_top_grid(n, 8, (n - 1) // 16, (n - 1) // 8)
    return AdjointWorkload(s, 1.0 / c_true**2, omega, h, (0, c0, c0), recv, dirs,
                           1e-3 * float(s.mean()))


def random_complex(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Standard complex normal array from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return z.astype(dtype)
