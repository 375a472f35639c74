"""Pins of the oracle's multigrid (paper section 3.4: damped Jacobi, full weighting,
trilinear interpolation, rediscretised coarse operators; Algorithm 1 applied
recursively as a V-cycle or an F-cycle)."""
import numpy as np
import pytest

import oracle as O
from oracle.discretization import DIRICHLET, SOMMERFELD, Level, boundary_directions, unknown_mask
from oracle.multigrid import build_hierarchy, coarsen_shape, fcycle, level_shapes, vcycle

from test_oracle_operator import sine_eigenvalue, sine_mode


def coords(shape, h):
    z, y, x = np.meshgrid(*[np.arange(m) * h for m in shape], indexing="ij")
    return z, y, x


@pytest.mark.parametrize("mode", [(1, 1, 1), (2, 3, 1), (5, 5, 6)])
def test_jacobi_sine_mode_amplification(mode):
    """Closed form: one damped-Jacobi step with b = 0 multiplies phi by
    1 - omega (lambda - (1 + 0.5i) k^2) / (6/h^2 - (1 + 0.5i) k^2)."""
    n, k, w = 17, 6.0, 0.8
    h = 1.0 / (n - 1)
    lvl = Level((n, n, n), h, np.full((n, n, n), k), DIRICHLET)
    phi = sine_mode(n, *mode).astype(np.complex128)
    d = O.diag_M(lvl)
    u = O.jacobi_sweep(phi, np.zeros_like(phi), lvl, w / d)
    sig = (1 + 0.5j) * k * k
    g = 1 - w * (sine_eigenvalue(h, *mode) - sig) / (6 / h**2 - sig)
    assert np.abs(u - g * phi).max() <= 1e-13 * np.abs(phi).max()


def test_jacobi_fixed_point():
    shape = (9, 9, 9)
    rng = np.random.default_rng(0)
    lvl = Level(shape, 0.1, rng.uniform(1, 4, shape), SOMMERFELD)
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    b = O.apply_M(u, lvl)
    u2 = O.jacobi_sweep(u, b, lvl, 0.8 / O.diag_M(lvl))
    assert np.abs(u2 - u).max() <= 1e-13 * np.abs(u).max()


@pytest.mark.parametrize("beta", [(1.0, -0.5), (1.0, -1.0)])
def test_sommerfeld_jacobi_sweep_against_assembled_matrix(beta):
    """One damped-Jacobi step of the hierarchy's finest level (the diagonal the
    V-cycle uses) against u + omega (b - M u) / diag(M) with M assembled row by
    row from section 2.4 (faces, edges and corners of a Sommerfeld grid): a
    missing, sign-flipped or misplaced -2ik/h term in D fails it."""
    from test_oracle_operator import rowwise_assembly

    b1, b2 = beta
    shape = (5, 7, 9)
    rng = np.random.default_rng(12)
    k = rng.uniform(2.0, 9.0, shape)
    h = 0.05
    hier = build_hierarchy(k, h, SOMMERFELD, n_levels=2, beta1=b1, beta2=b2)
    lvl = hier.levels[0]
    M = rowwise_assembly(lvl, complex(b1, -b2))
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    b = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    got = O.jacobi_sweep(u, b, lvl, hier.omega / hier.diags[0], b1, b2)
    ref = u.ravel() + 0.8 * (b.ravel() - M @ u.ravel()) / M.diagonal()
    assert np.abs(got.ravel() - ref).max() <= 1e-13 * np.abs(ref).max()


def test_restriction_preserves_constants_everywhere_and_linears_inside():
    fine = (9, 13, 17)
    h = 0.1
    z, y, x = coords(fine, h)
    c = np.full(fine, 2.5 - 1.0j)
    assert np.abs(O.restrict_fw(c, SOMMERFELD) - (2.5 - 1.0j)).max() <= 1e-14
    lin = 1.0 + 2.0 * x - 3.0 * y + 0.5 * z
    zc, yc, xc = coords(coarsen_shape(fine), 2 * h)
    r = O.restrict_fw(lin, SOMMERFELD)
    expect = 1.0 + 2.0 * xc - 3.0 * yc + 0.5 * zc
    assert np.abs(r - expect)[1:-1, 1:-1, 1:-1].max() <= 1e-13


def test_restriction_of_quadratic():
    """FW(x^2) = x^2 + h^2/2 per axis at interior coarse nodes."""
    fine = (9, 9, 9)
    h = 0.25
    z, y, x = coords(fine, h)
    zc, yc, xc = coords(coarsen_shape(fine), 2 * h)
    r = O.restrict_fw(x**2 + y**2 + z**2, SOMMERFELD)
    expect = xc**2 + yc**2 + zc**2 + 3 * h**2 / 2
    assert np.abs(r - expect)[1:-1, 1:-1, 1:-1].max() <= 1e-13


def test_restriction_single_fine_delta_gives_full_weighting_stencil():
    """The 27 weights of the full-weighting stencil (8/4/2/1 over 64)."""
    fine = (9, 9, 9)
    coarse = coarsen_shape(fine)
    Rt = np.zeros((3, 3, 3))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                r = np.zeros(fine)
                r[4 + dz, 4 + dy, 4 + dx] = 1.0
                Rt[dz + 1, dy + 1, dx + 1] = O.restrict_fw(r, DIRICHLET)[2, 2, 2]
    w = np.array([1, 2, 1])
    assert np.array_equal(Rt * 64, np.einsum("i,j,k->ijk", w, w, w))
    assert coarse == (5, 5, 5)


def test_prolongation_reproduces_trilinear_functions():
    coarse = (4 + 1, 3, 6 + 1)
    H = 0.2
    zc, yc, xc = coords(coarse, H)
    f = lambda z, y, x: (1 + 2 * x) * (3 - y) * (0.5 + z) + x * y * z
    fine = tuple(2 * (m - 1) + 1 for m in coarse)
    zf, yf, xf = coords(fine, H / 2)
    p = O.prolong_trilinear(f(zc, yc, xc).astype(np.complex128), fine)
    assert np.abs(p - f(zf, yf, xf)).max() <= 1e-14


def test_prolongation_of_coarse_delta_is_the_interpolation_stencil():
    coarse = (5, 5, 5)
    e = np.zeros(coarse)
    e[2, 2, 2] = 1.0
    p = O.prolong_trilinear(e, (9, 9, 9))
    w = np.array([0.5, 1.0, 0.5])
    stencil = np.einsum("i,j,k->ijk", w, w, w)
    assert np.array_equal(p[3:6, 3:6, 3:6], stencil)
    assert np.count_nonzero(p) == 27


def test_restriction_is_scaled_adjoint_of_prolongation():
    """<R r, e> = 1/8 <r, P e> (Dirichlet, interior unknowns) and the same with
    the D weights 2^(-n_j) on both grids at Sommerfeld boundaries (mirror
    extension makes R = D_H^-1 (P^T / 8) D_h)."""
    rng = np.random.default_rng(3)
    fine = (9, 11, 13)
    coarse = coarsen_shape(fine)
    for bc in (DIRICHLET, SOMMERFELD):
        r = rng.standard_normal(fine) * unknown_mask(fine, bc)
        e = rng.standard_normal(coarse) * unknown_mask(coarse, bc)
        Dh = 2.0 ** (-boundary_directions(fine)) if bc == SOMMERFELD else 1.0
        DH = 2.0 ** (-boundary_directions(coarse)) if bc == SOMMERFELD else 1.0
        Rr = O.restrict_fw(r, bc) * unknown_mask(coarse, bc)
        lhs = np.sum(DH * Rr * e)
        rhs = np.sum(Dh * r * O.prolong_trilinear(e, fine)) / 8.0
        assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


def test_level_shapes():
    assert level_shapes((33, 33, 33)) == [(33,) * 3, (17,) * 3, (9,) * 3, (5,) * 3, (3,) * 3]
    assert level_shapes((257, 129, 129))[-1] == (5, 3, 3)
    assert len(level_shapes((257, 129, 129))) == 7
    assert len(level_shapes((513, 513, 513), n_levels=8)) == 8
    assert level_shapes((513, 513, 513), n_levels=8)[-1] == (5, 5, 5)
    # the paper's "stop at 17" rule reproduces its 17^3 and 41 x 41 x 13 grids (section 4.2, 5.1.2)
    assert level_shapes((65, 65, 65), rule="paper17")[-1] == (17, 17, 17)
    assert level_shapes((193, 641, 641), rule="paper17")[-1] == (13, 41, 41)
    with pytest.raises(ValueError):
        level_shapes((32, 33, 33))


def _dense(fn, shape_in, mask_in, mask_out):
    """Dense matrix of a linear map restricted to the unknowns."""
    idx_in = np.flatnonzero(mask_in.ravel())
    cols = []
    for j in idx_in:
        e = np.zeros(shape_in, dtype=np.complex128)
        e.ravel()[j] = 1.0
        cols.append(fn(e).ravel()[np.flatnonzero(mask_out.ravel())])
    return np.array(cols).T


@pytest.mark.parametrize("bc", [DIRICHLET, SOMMERFELD])
def test_vcycle_equals_explicit_matrix_composition(bc):
    """Two routes on a 9^3 grid (3 levels): the recursive matrix-free V(1,1) cycle
    against the matrix V_l = W + (I - W M_l)(W + P V_{l+1} R (I - M_l W)),
    W = omega D_l^-1, assembled from dense R, P, M_l, D_l and the exact coarse inverse."""
    n = 9
    rng = np.random.default_rng(4)
    k = rng.uniform(3.0, 8.0, (n, n, n))
    h = 1.0 / (n - 1)
    hier = build_hierarchy(k, h, bc)
    assert len(hier.levels) == 3
    mats = {}
    L = len(hier.levels)
    lv = hier.levels[L - 1]
    mc = unknown_mask(lv.shape, bc)
    Mc = _dense(lambda x: O.apply_M(x, lv), lv.shape, mc, mc)
    mats[L - 1] = np.linalg.inv(Mc)
    for l in range(L - 2, -1, -1):
        lv, lc = hier.levels[l], hier.levels[l + 1]
        mf, mcm = unknown_mask(lv.shape, bc), unknown_mask(lc.shape, bc)
        M = _dense(lambda x: O.apply_M(x, lv), lv.shape, mf, mf)
        # the Jacobi diagonal taken from the dense M itself, not from O.diag_M
        W = np.diag(0.8 / np.diag(M))
        R = _dense(lambda x: O.restrict_fw(x, bc), lv.shape, mf, mcm)
        P = _dense(lambda x: O.prolong_trilinear(x, lv.shape), lc.shape, mcm, mf)
        I = np.eye(M.shape[0])
        mats[l] = W + (I - W @ M) @ (W + P @ mats[l + 1] @ R @ (I - M @ W))
    mf = unknown_mask((n, n, n), bc)
    b = (rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))) * mf
    u = vcycle(b, hier)
    u_dense = mats[0] @ b[mf]
    assert np.abs(u[mf] - u_dense).max() <= 1e-12 * np.abs(u_dense).max()


def test_vcycle_is_linear():
    n = 17
    rng = np.random.default_rng(5)
    hier = build_hierarchy(rng.uniform(5, 12, (n, n, n)), 1 / 16, SOMMERFELD)
    x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    y = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    a, c = 0.3 - 1.2j, 2.0 + 0.5j
    lhs = vcycle(a * x + c * y, hier)
    rhs = a * vcycle(x, hier) + c * vcycle(y, hier)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_vcycle_batched_equals_single():
    n = 9
    rng = np.random.default_rng(6)
    hier = build_hierarchy(rng.uniform(5, 12, (n, n, n)), 1 / 8, SOMMERFELD)
    b = rng.standard_normal((3, n, n, n)) + 1j * rng.standard_normal((3, n, n, n))
    ub = vcycle(b, hier)
    for r in range(3):
        assert np.array_equal(ub[r], vcycle(b[r], hier))


def _contraction(n, iters=12):
    h = 1.0 / (n - 1)
    k = np.zeros((n, n, n))
    hier = build_hierarchy(k, h, DIRICHLET)
    lvl = hier.levels[0]
    mask = unknown_mask(lvl.shape, DIRICHLET)
    rng = np.random.default_rng(7)
    e = rng.standard_normal((n, n, n)) * mask + 0j
    # stationary iteration e <- e - V(A e) on A u = 0 (k = 0: A = M = -Laplace_h)
    norms = []
    for _ in range(iters):
        e = e - vcycle(O.apply_A(e, lvl), hier)
        norms.append(np.linalg.norm(e))
    return (norms[-1] / norms[-5]) ** 0.25


def test_vcycle_contracts_mesh_independently_for_k0():
    """k = 0 Dirichlet: u <- u + V(b - A u) converges with a factor that does not
    grow with the grid (textbook multigrid property)."""
    rhos = [_contraction(n) for n in (17, 33, 65)]
    assert all(r < 0.6 for r in rhos), rhos
    assert max(rhos) - min(rhos) < 0.05, rhos


def test_vcycle_mixed_precision_close_to_double():
    n = 33
    rng = np.random.default_rng(8)
    k = rng.uniform(5, 10, (n, n, n))
    h64 = build_hierarchy(k, 1 / 32, SOMMERFELD)
    h32 = build_hierarchy(k, 1 / 32, SOMMERFELD, dtype=np.complex64)
    b = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    u64 = vcycle(b, h64)
    u32 = vcycle(b.astype(np.complex64), h32)
    assert u32.dtype == np.complex64
    assert np.linalg.norm(u32 - u64) <= 1e-5 * np.linalg.norm(u64)


def _two_grid_mats(hier, bc, coarse_inv, l):
    """Dense level-l pieces: M_l, W = omega D_l^-1, R, P and the V-type two-grid matrix
    W + (I - W M)(W + P C R (I - M W)) for a given coarse solver matrix C."""
    lv, lc = hier.levels[l], hier.levels[l + 1]
    mf, mcm = unknown_mask(lv.shape, bc), unknown_mask(lc.shape, bc)
    M = _dense(lambda x: O.apply_M(x, lv), lv.shape, mf, mf)
    W = np.diag(0.8 / np.diag(M))  # from the dense M, not from O.diag_M
    R = _dense(lambda x: O.restrict_fw(x, bc), lv.shape, mf, mcm)
    P = _dense(lambda x: O.prolong_trilinear(x, lv.shape), lc.shape, mcm, mf)
    I = np.eye(M.shape[0])
    return M, W + (I - W @ M) @ (W + P @ coarse_inv @ R @ (I - M @ W))


def test_fcycle_with_two_levels_is_the_vcycle():
    """With one coarse level the coarse solve is exact, so no extra cycle is made."""
    n = 9
    rng = np.random.default_rng(41)
    for bc in (DIRICHLET, SOMMERFELD):
        hier = build_hierarchy(rng.uniform(3, 8, (n, n, n)), 1 / 8, bc, n_levels=2)
        b = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
        b = b * unknown_mask((n, n, n), bc)
        assert np.array_equal(fcycle(b, hier), vcycle(b, hier))


@pytest.mark.parametrize("bc", [DIRICHLET, SOMMERFELD])
def test_fcycle_with_three_levels_is_the_wcycle(bc):
    """Three levels: the F-cycle visits the middle level twice, which is the W-cycle
    (two two-grid iterations on the middle level, the second started from the first's
    result).  Assembled from dense matrices: C_1 = 2 B_1 - B_1 M_1 B_1, with B_1 the
    middle level's two-grid matrix over the exact coarsest inverse."""
    n = 9
    rng = np.random.default_rng(42)
    k = rng.uniform(3.0, 8.0, (n, n, n))
    hier = build_hierarchy(k, 1.0 / (n - 1), bc)
    assert len(hier.levels) == 3
    lv = hier.levels[2]
    mc = unknown_mask(lv.shape, bc)
    inv2 = np.linalg.inv(_dense(lambda x: O.apply_M(x, lv), lv.shape, mc, mc))
    M1, B1 = _two_grid_mats(hier, bc, inv2, 1)
    C1 = 2 * B1 - B1 @ M1 @ B1
    _, F0 = _two_grid_mats(hier, bc, C1, 0)
    _, V0 = _two_grid_mats(hier, bc, B1, 0)
    mf = unknown_mask((n, n, n), bc)
    b = (rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))) * mf
    u = fcycle(b, hier)
    ref = F0 @ b[mf]
    assert np.abs(u[mf] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(u[~mf]).max() == 0 if bc == DIRICHLET else True
    # and it is not the V-cycle
    assert np.abs(u[mf] - V0 @ b[mf]).max() > 1e-3 * np.abs(ref).max()


def test_fcycle_is_linear_and_batched():
    n = 17
    rng = np.random.default_rng(43)
    hier = build_hierarchy(rng.uniform(5, 12, (n, n, n)), 1 / 16, SOMMERFELD)
    x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    y = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    a, c = 0.3 - 1.2j, 2.0 + 0.5j
    lhs = fcycle(a * x + c * y, hier)
    rhs = a * fcycle(x, hier) + c * fcycle(y, hier)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()
    ub = fcycle(np.stack([x, y]), hier)
    assert np.array_equal(ub[0], fcycle(x, hier)) and np.array_equal(ub[1], fcycle(y, hier))


def _wcycle(b, hier, level=0):
    """W(1,1) cycle from zero, composed here from the oracle's level primitives:
    the coarse error equation gets two cycles, the second on the first's residual."""
    from oracle.multigrid import coarse_solve, jacobi_sweep, prolong_trilinear, restrict_fw

    lvl = hier.levels[level]
    if level == len(hier.levels) - 1:
        return coarse_solve(b, hier)
    wd = hier.omega / hier.diags[level]
    u = jacobi_sweep(np.zeros_like(b), b, lvl, wd, hier.beta1, hier.beta2)
    coarse = hier.levels[level + 1]
    mc, mf = unknown_mask(coarse.shape, lvl.bc), unknown_mask(lvl.shape, lvl.bc)
    bc_ = restrict_fw(b - O.apply_M(u, lvl, hier.beta1, hier.beta2), lvl.bc) * mc
    e = _wcycle(bc_, hier, level + 1)
    e = e + _wcycle(bc_ - O.apply_M(e, coarse, hier.beta1, hier.beta2), hier, level + 1)
    u = jacobi_sweep(u + prolong_trilinear(e, lvl.shape), b, lvl, wd, hier.beta1, hier.beta2)
    return u * mf


def _contraction_of(cycle, n, iters=12):
    k = np.zeros((n, n, n))
    hier = build_hierarchy(k, 1.0 / (n - 1), DIRICHLET)
    lvl = hier.levels[0]
    mask = unknown_mask(lvl.shape, DIRICHLET)
    e = np.random.default_rng(7).standard_normal((n, n, n)) * mask + 0j
    norms = []
    for _ in range(iters):
        e = (e - cycle(O.apply_A(e, lvl), hier)) * mask
        norms.append(np.linalg.norm(e))
    return (norms[-1] / norms[-5]) ** 0.25


def test_fcycle_contraction_between_w_and_v_for_k0():
    """k = 0 Dirichlet on 33^3 (5 levels): the F-cycle's asymptotic contraction lies
    between the W-cycle's and the V-cycle's (textbook ordering), and does not grow
    from 17^3 to 33^3."""
    rv = _contraction_of(vcycle, 33)
    rf = _contraction_of(fcycle, 33)
    rw = _contraction_of(_wcycle, 33)
    assert rw <= rf + 1e-3 and rf < rv, (rw, rf, rv)
    rf17 = _contraction_of(fcycle, 17)
    assert rf <= rf17 + 0.05, (rf17, rf)


@pytest.mark.parametrize("bc", [DIRICHLET, SOMMERFELD])
def test_coarse_gmres_reaches_the_exact_coarse_solution(bc):
    """The paper's coarsest-grid solve (full GMRES to relative residual 1e-11,
    end of section 3.4.5 and section 5) against the sparse LU solve of the same
    coarsest M: on the 17^3 coarsest grid of the closed-off configuration
    (k = 40, h = 1/16 there) and a heterogeneous k, the GMRES result lies
    within the residual bound times a small condition number of the exact
    solution, and its true residual meets 1e-11."""
    from oracle.discretization import apply_M
    from oracle.multigrid import coarse_gmres, coarse_solve

    for k in (np.full((33, 33, 33), 40.0), np.random.default_rng(3).uniform(20.0, 60.0, (33, 33, 33))):
        exact = build_hierarchy(k, 1 / 32, bc, n_levels=2)
        itv = build_hierarchy(k, 1 / 32, bc, n_levels=2, coarse="gmres")
        assert exact.coarsest.shape == (17, 17, 17)
        mask = unknown_mask((17, 17, 17), bc)
        rng = np.random.default_rng(4)
        b = (rng.standard_normal((17, 17, 17)) + 1j * rng.standard_normal((17, 17, 17))) * mask
        e_lu = coarse_solve(b, exact)
        e_gm, steps = coarse_gmres(b, itv)
        assert 10 <= steps <= 200
        res = np.linalg.norm((b - apply_M(e_gm, itv.coarsest)) * mask) / np.linalg.norm(b)
        assert res <= 1.5e-11, res
        assert np.linalg.norm(e_gm - e_lu) / np.linalg.norm(e_lu) <= 1e-9
        assert np.all(e_gm[~mask.astype(bool)] == 0)


@pytest.mark.parametrize("bc", [DIRICHLET, SOMMERFELD])
def test_cycles_with_coarse_gmres_equal_cycles_with_the_exact_coarse_solve(bc):
    """V- and F-cycles whose coarsest level is solved by GMRES to 1e-11 agree
    with the exact-solve cycles to about that tolerance (three levels down to
    9^3, two right-hand sides; the mixed form solves its coarsest level in
    complex128 too)."""
    shape = (33, 33, 33)
    k = np.random.default_rng(5).uniform(4.0, 12.0, shape)
    rng = np.random.default_rng(6)
    r = (rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape)) * unknown_mask(shape, bc)
    for dtype, tol in ((np.complex128, 1e-10), (np.complex64, 1e-5)):
        exact = build_hierarchy(k, 1 / 32, bc, n_levels=3, dtype=dtype)
        itv = build_hierarchy(k, 1 / 32, bc, n_levels=3, dtype=dtype, coarse="gmres")
        for cyc in (vcycle, fcycle):
            za = cyc(r.astype(dtype), exact)
            zb = cyc(r.astype(dtype), itv)
            assert zb.dtype == dtype
            assert np.abs(zb - za).max() <= tol * np.abs(za).max(), (dtype, cyc.__name__)
