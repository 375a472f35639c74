"""Pins of the oracle's operators A_h, M_h (paper section 2.4, eq. Helmstencil and
eq. elimination; section 3.3 eq. preconditioner) against closed forms and invariants."""
import numpy as np
import pytest

import oracle as O
from oracle.discretization import DIRICHLET, SOMMERFELD, Level, boundary_directions


def sine_mode(n, p, q, r):
    t = np.linspace(0.0, 1.0, n)
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return np.sin(p * np.pi * x) * np.sin(q * np.pi * y) * np.sin(r * np.pi * z)


def sine_eigenvalue(h, p, q, r):
    s = lambda m: np.sin(m * np.pi * h / 2) ** 2
    return 4.0 / h**2 * (s(p) + s(q) + s(r))


@pytest.mark.parametrize("n", [9, 17])
@pytest.mark.parametrize("mode", [(1, 1, 1), (1, 2, 4), (3, 1, 2), (7, 7, 7)])
def test_dirichlet_sine_modes_are_eigenvectors(n, mode):
    """Closed form: A phi = (lambda - k^2) phi, M phi = (lambda - (1 + 0.5i) k^2) phi."""
    if max(mode) >= n - 1:
        pytest.skip("mode not resolved")
    h = 1.0 / (n - 1)
    k = 7.5
    lvl = Level((n, n, n), h, np.full((n, n, n), k), DIRICHLET)
    phi = sine_mode(n, *mode).astype(np.complex128)
    lam = sine_eigenvalue(h, *mode)
    Aphi = O.apply_A(phi, lvl)
    Mphi = O.apply_M(phi, lvl)
    scale = np.abs(lam) * np.abs(phi).max()
    assert np.abs(Aphi - (lam - k * k) * phi).max() <= 1e-13 * scale
    assert np.abs(Mphi - (lam - (1 + 0.5j) * k * k) * phi).max() <= 1e-13 * scale


def _random_level(shape, bc, seed=0):
    rng = np.random.default_rng(seed)
    h = 0.05
    k = rng.uniform(2.0, 9.0, size=shape)
    return Level(shape, h, k, bc)


def test_sommerfeld_D_scaled_operator_is_complex_symmetric():
    """Invariant: x^T (D A) y = y^T (D A) x with D_j = 2^(-n_j) (bilinear, no conjugation).

    A wrong mirror coefficient at faces, edges or corners breaks it."""
    shape = (5, 7, 9)
    lvl = _random_level(shape, SOMMERFELD)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    y = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    D = 2.0 ** (-boundary_directions(shape))
    for op in (O.apply_A, O.apply_M):
        lhs = np.sum(x * D * op(y, lvl))
        rhs = np.sum(y * D * op(x, lvl))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # and the undscaled operator is NOT symmetric (the paper's "symmetric" needs D)
    lhs = np.sum(x * O.apply_A(y, lvl))
    rhs = np.sum(y * O.apply_A(x, lvl))
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)


def test_dirichlet_operator_is_symmetric():
    shape = (7, 9, 11)
    lvl = _random_level(shape, DIRICHLET)
    mask = O.unknown_mask(shape, DIRICHLET)
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * mask
    y = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * mask
    lhs = np.sum(x * O.apply_A(y, lvl))
    rhs = np.sum(y * O.apply_A(x, lvl))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_sommerfeld_boundary_absorption_identity():
    """Im(x^H D A x) = -sum_j D_j n_j (2 k_j / h) |x_j|^2.

    D*(-Laplace_h - k^2) is real symmetric, so the imaginary part of the D-weighted
    energy comes only from the ghost-elimination terms -2ik/h: this pins their
    sign, the factor 2 and which node's k is used."""
    shape = (6 + 1, 5, 9)
    lvl = _random_level(shape, SOMMERFELD, seed=3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    nj = boundary_directions(shape)
    D = 2.0 ** (-nj)
    energy = np.sum(np.conj(x) * D * O.apply_A(x, lvl))
    expect = -np.sum(D * nj * 2 * lvl.k / lvl.h * np.abs(x) ** 2)
    assert abs(energy.imag - expect) <= 1e-12 * abs(expect)


def test_sommerfeld_zero_wavenumber_annihilates_constants():
    """With k = 0 the eliminated ghost equals the mirror (Neumann); -Laplace_h of a
    constant vanishes at every node, faces, edges and corners included."""
    shape = (5, 7, 9)
    lvl = Level(shape, 0.1, np.zeros(shape), SOMMERFELD)
    y = O.apply_A(np.full(shape, 3.0 + 1.0j), lvl)
    assert np.abs(y).max() <= 1e-12


def test_matrix_free_equals_rowwise_assembly():
    """Row-by-row sparse assembly of section 2.4 (7-point stencil, eliminated ghost
    points: the inward neighbour's coupling doubles and the diagonal gains
    -2ik/h per missing neighbour) against the matrix-free apply of Algorithm 2."""
    import scipy.sparse as sp

    shape = (4 + 1, 3 + 2, 7)
    lvl = _random_level(shape, SOMMERFELD, seed=5)
    nz, ny, nx = shape
    h = lvl.h
    idx = np.arange(nz * ny * nx).reshape(shape)
    rows, cols, vals = [], [], []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                j = idx[z, y, x]
                kk = lvl.k[z, y, x]
                diag = 6.0 / h**2 - kk**2
                for axis, pos, n in ((0, z, nz), (1, y, ny), (2, x, nx)):
                    for step in (-1, 1):
                        q = pos + step
                        if 0 <= q < n:
                            nb = [z, y, x]
                            nb[axis] = q
                        else:
                            nb = [z, y, x]
                            nb[axis] = pos - step
                            diag += -2j * kk / h
                        rows.append(j)
                        cols.append(idx[tuple(nb)])
                        vals.append(-1.0 / h**2)
                rows.append(j)
                cols.append(j)
                vals.append(diag)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(idx.size, idx.size))
    rng = np.random.default_rng(6)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    y = O.apply_A(x, lvl)
    assert np.abs(A @ x.ravel() - y.ravel()).max() <= 1e-13 * np.abs(y).max()


def test_single_precision_apply_tracks_double():
    shape = (9, 9, 9)
    lvl = _random_level(shape, SOMMERFELD, seed=7)
    lvl32 = Level(shape, lvl.h, lvl.k.astype(np.float32), SOMMERFELD)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    y64 = O.apply_M(x, lvl)
    y32 = O.apply_M(x.astype(np.complex64), lvl32)
    assert y32.dtype == np.complex64
    assert np.linalg.norm(y32 - y64) <= 1e-5 * np.linalg.norm(y64)


def test_point_source_rhs():
    b = O.point_source_rhs((5, 5, 5), 0.25, [(2, 2, 2), (0, 1, 3)])
    assert b.shape == (2, 5, 5, 5)
    assert b[0, 2, 2, 2] == 64.0 and b[1, 0, 1, 3] == 64.0
    assert np.count_nonzero(b) == 2


def test_closed_off_exact_solution_has_second_order_truncation():
    """A_h u* - b_h = O(h^2) at interior nodes for the closed-off problem (section 2.1)."""
    errs = []
    for n in (17, 33, 65):
        lvl, b, uex = O.closed_off_problem(n, 10.0)
        r = O.apply_A(uex.astype(np.complex128), lvl) - b
        errs.append(np.abs(r).max())
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.6 < q < 4.4 for q in ratios), ratios
