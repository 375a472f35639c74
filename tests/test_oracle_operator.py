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


def rowwise_assembly(lvl, shift=1.0):
    """Sparse matrix of -Laplace_h - shift k^2 I assembled row by row from section
    2.4 (7-point stencil; at a Sommerfeld boundary the ghost point of eq.
    elimination is replaced by mirror + 2 h i k u_j, so the inward neighbour's
    coupling doubles and the diagonal gains -2ik/h per missing neighbour).
    Dirichlet: rows and columns of the interior unknowns only, indexed like the
    full grid (boundary rows are empty)."""
    import scipy.sparse as sp

    nz, ny, nx = lvl.shape
    h = lvl.h
    idx = np.arange(nz * ny * nx).reshape(lvl.shape)
    rows, cols, vals = [], [], []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                j = idx[z, y, x]
                kk = lvl.k[z, y, x]
                interior = 0 < z < nz - 1 and 0 < y < ny - 1 and 0 < x < nx - 1
                if lvl.bc == DIRICHLET and not interior:
                    continue
                diag = 6.0 / h**2 - shift * kk**2
                for axis, pos, n in ((0, z, nz), (1, y, ny), (2, x, nx)):
                    for step in (-1, 1):
                        nb = [z, y, x]
                        q = pos + step
                        if 0 <= q < n:
                            nb[axis] = q
                            if lvl.bc == DIRICHLET and not (0 < q < n - 1):
                                continue  # a boundary neighbour carries g = 0
                        else:
                            nb[axis] = pos - step
                            diag += -2j * kk / h
                        rows.append(j)
                        cols.append(idx[tuple(nb)])
                        vals.append(-1.0 / h**2)
                rows.append(j)
                cols.append(j)
                vals.append(diag)
    return sp.csr_matrix((vals, (rows, cols)), shape=(idx.size, idx.size))


@pytest.mark.parametrize("op", ["A", "M"])
@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
def test_matrix_free_equals_rowwise_assembly(op, bc):
    """Row-by-row sparse assembly of section 2.4 (and of M_h with the shift
    (1 + 0.5i) k^2 of section 3.3 in the volume term only) against the
    matrix-free apply of Algorithm 2."""
    shape = (4 + 1, 3 + 2, 7)
    lvl = _random_level(shape, bc, seed=5)
    shift = 1.0 if op == "A" else (1 + 0.5j)
    A = rowwise_assembly(lvl, shift)
    rng = np.random.default_rng(6)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * O.unknown_mask(shape, bc)
    y = O.apply_A(x, lvl) if op == "A" else O.apply_M(x, lvl)
    assert np.abs(A @ x.ravel() - y.ravel()).max() <= 1e-13 * np.abs(y).max()


@pytest.mark.parametrize("beta", [(1.0, -0.5), (1.0, -1.0), (0.7, 0.3)])
def test_diag_M_equals_rowwise_diagonal(beta):
    """The Jacobi diagonal D = diag(M_h) (section 3.4.1) against the diagonal of the
    row-wise assembled M_h: on a Sommerfeld grid every node kind occurs (interior,
    faces n_j = 1, edges n_j = 2, corners n_j = 3), each with its -2ik/h per
    missing neighbour; Dirichlet interior rows have no boundary term."""
    b1, b2 = beta
    shift = complex(b1, -b2)
    shape = (5, 6, 7)
    for bc in (SOMMERFELD, DIRICHLET):
        lvl = _random_level(shape, bc, seed=9)
        ref = rowwise_assembly(lvl, shift).diagonal().reshape(shape)
        d = O.diag_M(lvl, b1, b2)
        mask = O.unknown_mask(shape, bc)
        assert np.abs(d[mask] - ref[mask]).max() <= 1e-14 * np.abs(ref[mask]).max()
        if bc == SOMMERFELD:
            nj = boundary_directions(shape)
            assert {0, 1, 2, 3} <= set(np.unique(nj))
            # the boundary term is what separates the node kinds: with it removed
            # (or its sign flipped) every boundary row would differ
            plain = 6.0 / lvl.h**2 - shift * lvl.k**2
            assert np.all(np.abs(d - plain)[nj > 0] > 1.0 / lvl.h)


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
