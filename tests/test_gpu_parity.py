"""GPU parity: every C-ABI entry point against the CPU oracle on the same seeded inputs.

Tolerances (relative to the largest entry of the reference):
* operator and shifted operator, complex128: 1e-13 (FMA contraction and
  summation order differ from NumPy; the stencil has ~10 terms);
* one V-cycle, complex128: 1e-12; mixed (complex64 V-cycle): 1e-5 against the
  oracle's complex64 V-cycle and against its complex128 V-cycle;
* solve: true residual under the oracle's operator <= rtol; at rtol 1e-10 both
  sides agree to 1e-6; fixed-iteration iterates agree to 1e-9 (mixed: 2e-6);
* Bi-CGSTAB counts may differ by rounding: |d iters| <= max(2, 5 %).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.discretization import DIRICHLET, SOMMERFELD, Level, unknown_mask
from oracle.multigrid import build_hierarchy, vcycle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver(shape, h, bc, **kw):
    from paper_2308_06085_amd import Solver

    return Solver(shape, h, bc=bc, **kw)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def hetero_k(shape, seed, lo=4.0, hi=12.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


# shapes: several workgroups per plane, ragged last workgroup, non-cubic, and
# level counts from 2 to 5
SHAPES = [(9, 9, 9), (17, 9, 33), (33, 17, 17), (5, 9, 65), (9, 65, 129), (33, 97, 41)]


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("shape", SHAPES)
def test_apply_operator_and_shifted(bc, shape):
    h = 1.0 / (max(shape) - 1)
    k = hetero_k(shape, 1)
    lvl = Level(shape, h, k, bc)
    x = W.random_complex((2,) + shape, seed=2)
    s = _solver(shape, h, bc, nrhs_max=2)
    s.set_model(dev(k))
    y = host(s.apply_operator(dev(x)))
    ym = host(s.apply_shifted(dev(x)))
    ref = O.apply_A(x, lvl)
    refm = O.apply_M(x, lvl)
    if bc == DIRICHLET:
        assert not y[:, 0].any() and not y[:, :, :, -1].any()
    assert relerr(y, ref) <= 1e-13
    assert relerr(ym, refm) <= 1e-13


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
def test_apply_tiles_and_zblocks(bc):
    """The operator apply on planes that give one tile five nodes wide, a
    ragged last tile in x or y and four tiles across a row (x-y tiles of at
    most 256 nodes with a one-node halo): every result matches the oracle,
    and does not depend on the z-planes per workgroup, bit for bit (each
    node's arithmetic is fixed)."""
    for shape in [(5, 5, 5), (9, 5, 5), (9, 17, 193), (5, 257, 5), (9, 33, 97)]:
        h = 1.0 / (max(shape) - 1)
        k = hetero_k(shape, 5)
        lvl = Level(shape, h, k, bc)
        x = W.random_complex(shape, seed=6)
        s = _solver(shape, h, bc)
        s.set_model(dev(k))
        y0 = host(s.apply_operator(dev(x)))[0]
        assert relerr(y0, O.apply_A(x, lvl)) <= 1e-13, shape
        for zb in (1, 2, 3, 7):
            s.set_option("zb", zb)
            assert np.array_equal(host(s.apply_operator(dev(x)))[0], y0), (shape, zb)
        s.close()


def test_dirichlet_inputs_on_the_boundary_are_ignored():
    shape = (9, 9, 9)
    h = 1 / 8
    k = hetero_k(shape, 3)
    x = W.random_complex(shape, seed=4)
    s = _solver(shape, h, DIRICHLET)
    s.set_model(dev(k))
    y1 = host(s.apply_operator(dev(x)))
    xz = x * unknown_mask(shape, DIRICHLET)
    y2 = host(s.apply_operator(dev(xz)))
    assert np.array_equal(y1, y2)


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("shape", SHAPES)
def test_vcycle_fp64(bc, shape):
    h = 1.0 / (max(shape) - 1)
    k = hetero_k(shape, 5)
    hier = build_hierarchy(k, h, bc)
    r = W.random_complex((2,) + shape, seed=6) * unknown_mask(shape, bc)
    s = _solver(shape, h, bc, nrhs_max=2)
    assert s.level_shapes() == [lv.shape for lv in hier.levels]
    s.set_model(dev(k))
    z = host(s.apply_vcycle(dev(r)))
    ref = vcycle(r, hier)
    assert relerr(z, ref) <= 1e-12


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
def test_vcycle_mixed(bc):
    shape = (17, 33, 33)
    h = 1 / 32
    k = hetero_k(shape, 7)
    h64 = build_hierarchy(k, h, bc)
    h32 = build_hierarchy(k, h, bc, dtype=np.complex64)
    r = W.random_complex(shape, seed=8) * unknown_mask(shape, bc)
    s = _solver(shape, h, bc, prec="mixed")
    s.set_model(dev(k))
    z = host(s.apply_vcycle(dev(r)))[0]
    ref32 = vcycle(r.astype(np.complex64), h32).astype(np.complex128)
    ref64 = vcycle(r, h64)
    assert relerr(z, ref32) <= 1e-5
    assert relerr(z, ref64) <= 1e-5


def test_explicit_level_count_matches_oracle():
    shape = (33, 33, 33)
    h = 1 / 32
    k = hetero_k(shape, 9)
    hier = build_hierarchy(k, h, SOMMERFELD, n_levels=3)
    s = _solver(shape, h, SOMMERFELD, n_levels=3)
    assert s.level_shapes() == [lv.shape for lv in hier.levels]
    s.set_model(dev(k))
    r = W.random_complex(shape, seed=10)
    assert relerr(host(s.apply_vcycle(dev(r)))[0], vcycle(r, hier)) <= 1e-12


def _random_shapes(n, seed):
    """Seeded grid sizes m 2^j + 1 per axis (m = 1, 3, 5, 7, so the hierarchy
    coarsens down to a small grid) with 1..4 right-hand sides: tile splits,
    ragged tiles and down-pass regions vary from case to case."""
    sizes = [9, 13, 17, 21, 25, 29, 33, 41, 49, 57, 65]
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        shape = tuple(int(rng.choice(sizes)) for _ in range(3))
        out.append((shape, int(rng.integers(1, 5))))
    return out


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("shape,nrhs", _random_shapes(6, 13))
def test_vcycle_random_shapes(bc, shape, nrhs):
    h = 1.0 / (max(shape) - 1)
    k = hetero_k(shape, 14)
    hier = build_hierarchy(k, h, bc)
    r = W.random_complex((nrhs,) + shape, seed=15) * unknown_mask(shape, bc)
    s = _solver(shape, h, bc, nrhs_max=nrhs)
    assert s.level_shapes() == [lv.shape for lv in hier.levels]
    s.set_model(dev(k))
    assert relerr(host(s.apply_vcycle(dev(r))), vcycle(r, hier)) <= 1e-12, (shape, nrhs)
    s.close()
    m = _solver(shape, h, bc, nrhs_max=nrhs, prec="mixed")
    m.set_model(dev(k))
    h32 = build_hierarchy(k, h, bc, dtype=np.complex64)
    ref32 = vcycle(r.astype(np.complex64), h32).astype(np.complex128)
    assert relerr(host(m.apply_vcycle(dev(r))), ref32) <= 1e-5, (shape, nrhs)
    m.close()


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("shape,nrhs", _random_shapes(6, 16))
def test_apply_random_shapes(bc, shape, nrhs):
    h = 1.0 / (max(shape) - 1)
    k = hetero_k(shape, 17)
    lvl = Level(shape, h, k, bc)
    x = W.random_complex((nrhs,) + shape, seed=18)
    s = _solver(shape, h, bc, nrhs_max=nrhs)
    s.set_model(dev(k))
    assert relerr(host(s.apply_operator(dev(x))), O.apply_A(x, lvl)) <= 1e-13, (shape, nrhs)
    assert relerr(host(s.apply_shifted(dev(x))), O.apply_M(x, lvl)) <= 1e-13, (shape, nrhs)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_down_pass_regions_batched_equals_single(prec):
    """The one-plane down pass stages 1280, 512 or 256 fine nodes per
    workgroup, chosen by the launch's size: on this grid's finest level 512
    for one right-hand side, 256 for four and 1280 for sixteen.  Each node's
    arithmetic is the same, so batched V-cycles equal the single ones bit for
    bit; one of them is checked against the oracle."""
    shape, h = (129, 65, 65), 1 / 64
    k = hetero_k(shape, 11)
    r = W.random_complex((16,) + shape, seed=12)
    s = _solver(shape, h, SOMMERFELD, nrhs_max=16, prec=prec)
    assert s.get_option("zb_down:0") == 1
    s.set_model(dev(k))
    single = [host(s.apply_vcycle(dev(r[i])))[0] for i in range(4)]
    b4 = host(s.apply_vcycle(dev(r[:4])))
    b16 = host(s.apply_vcycle(dev(r)))
    for i in range(4):
        assert np.array_equal(b4[i], single[i]) and np.array_equal(b16[i], single[i]), i
    if prec == "fp64":
        ref = vcycle(r[0], build_hierarchy(k, h, SOMMERFELD))
        assert relerr(single[0], ref) <= 1e-12
    else:
        ref = vcycle(r[0].astype(np.complex64), build_hierarchy(k, h, SOMMERFELD, dtype=np.complex64))
        assert relerr(single[0], ref.astype(np.complex128)) <= 1e-5
    s.close()


# --------------------------------------------------------------------------
# solves
# --------------------------------------------------------------------------
def _oracle_solve(wl, b, tol, **kw):
    lvl = Level(wl.shape, wl.h, wl.k, wl.bc)
    hier = build_hierarchy(wl.k, wl.h, wl.bc, n_levels=wl.n_levels)
    return O.bicgstab(lambda x: O.apply_A(x, lvl), lambda r: vcycle(r, hier), b, tol=tol, **kw), lvl


def test_solve_small_dirichlet_cube_parity():
    """k = 10 on the 33^3 unit cube, Dirichlet, centre source, FP64."""
    wl = W.constant_cube(33, 10.0, DIRICHLET)
    b = O.point_source_rhs(wl.shape, wl.h, wl.sources)[0]
    s = _solver(wl.shape, wl.h, DIRICHLET)
    s.set_model(dev(wl.k))
    s.set_point_sources(wl.sources)
    x, st = s.solve(rtol=1e-6)
    x = host(x)[0]
    ref, lvl = _oracle_solve(wl, b, 1e-6)
    true_rel = np.linalg.norm(b - O.apply_A(x, lvl)) / np.linalg.norm(b)
    assert st[0].status == "HH_OK" and true_rel <= 1e-6
    assert abs(st[0].iterations - ref.iterations) <= max(2, 0.05 * ref.iterations)
    assert abs(st[0].relres_true - true_rel) <= 1e-9
    # tight solves agree
    x10, st10 = s.solve(rtol=1e-10)
    ref10, _ = _oracle_solve(wl, b, 1e-10)
    assert np.linalg.norm(host(x10)[0] - ref10.x) <= 1e-6 * np.linalg.norm(ref10.x)


@pytest.mark.parametrize("steps", [1, 2, 5])
def test_fixed_iteration_iterates(steps):
    shape = (17, 17, 33)
    h = 1 / 16
    k = hetero_k(shape, 11, 6.0, 14.0)
    wl = W.Workload(k, h, SOMMERFELD, [(8, 8, 16)], 0, "hetero")
    b = O.point_source_rhs(shape, h, wl.sources)[0]
    ref, _ = _oracle_solve(wl, b, 1e-6, fixed_iterations=steps)
    s = _solver(shape, h, SOMMERFELD)
    s.set_model(dev(k))
    s.set_point_sources(wl.sources)
    x, st = s.solve(rtol=1e-14, maxit=steps)
    assert st[0].status == "HH_ERR_NOT_CONVERGED" and st[0].iterations == steps
    assert relerr(host(x)[0], ref.x) <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_check_window_does_not_change_the_solution(prec):
    """The solve updates x every second step and replays an even/odd pair of
    steps per graph launch, so host checks every 1 or 3 steps round up to whole
    pairs; steps after a right-hand side stops are gated off, so the window
    changes neither the solution (bit for bit) nor the step count.  Two
    right-hand sides stop at different steps.  The mixed form's restarts at
    every power of ten run at the head of the next even step, inside a window
    or, when the decision falls on a window's last step, at the host check:
    the same arithmetic either way."""
    shape = (17, 17, 33)
    h = 1 / 16
    k = hetero_k(shape, 11, 6.0, 14.0)
    s = _solver(shape, h, SOMMERFELD, prec=prec, nrhs_max=2)
    s.set_model(dev(k))
    b = np.stack([O.point_source_rhs(shape, h, [(8, 8, 16)])[0], W.random_complex(shape, seed=29)])
    s.set_sources(dev(b))
    ref, st_ref = s.solve(rtol=1e-6)
    ref = host(ref)
    assert st_ref[0].iterations != st_ref[1].iterations
    if prec == "mixed":
        assert min(t.restarts for t in st_ref) >= 3, [t.restarts for t in st_ref]
    for ce in (1, 3, 4, 8):
        s.set_option("check_every", ce)
        x, st = s.solve(rtol=1e-6)
        assert np.array_equal(host(x), ref), ce
        assert [t.iterations for t in st] == [t.iterations for t in st_ref], ce
    s.close()


@pytest.mark.parametrize("bc,steps,restart",
                         [(bc, st, rs) for bc in (SOMMERFELD, DIRICHLET) for st in (1, 2, 5) for rs in (0, 1)]
                         + [(SOMMERFELD, 9, 1)])
def test_fixed_iteration_iterates_mixed(bc, steps, restart):
    """The mixed solve (complex64 V-cycle and shadow residual r_hat = r_0
    rounded to complex64, complex128 Krylov vectors) against the oracle's
    Bi-CGSTAB with the same precisions: fixed-step iterates agree to the
    complex64 V-cycle's tolerance, with and without the restarts from x at
    every power of ten of the residual (the mixed form's default).  With
    Sommerfeld boundaries the residual passes 0.1 after step 2 and 0.01 after
    step 7, so 5 and 9 steps include one and two restarts.  Without restarts
    the iterates grow sensitive to the rounding of the preconditioner beyond
    about six steps here (a relative change of 1e-7 in its output moves the
    9-step iterate by 1e-4 in the oracle, by 3e-8 with restarts)."""
    shape = (17, 17, 33)
    h = 1 / 16
    k = hetero_k(shape, 11, 6.0, 14.0)
    src = [(8, 8, 16)]
    b = O.point_source_rhs(shape, h, src)[0]
    lvl = Level(shape, h, k, bc)
    h32 = build_hierarchy(k, h, bc, dtype=np.complex64)
    ref = O.bicgstab(lambda v: O.apply_A(v, lvl),
                     lambda v: vcycle(v.astype(np.complex64), h32).astype(np.complex128), b,
                     fixed_iterations=steps, shadow_dtype=np.complex64, restart_decade=bool(restart))
    s = _solver(shape, h, bc, prec="mixed")
    assert s.get_option("restart_decade") == 1
    s.set_option("restart_decade", restart)
    s.set_model(dev(k))
    s.set_point_sources(src)
    x, st = s.solve(rtol=1e-14, maxit=steps)
    assert st[0].status == "HH_ERR_NOT_CONVERGED" and st[0].iterations == steps
    # measured 1e-8 .. 2.4e-7 (the two complex64 V-cycles round differently)
    assert relerr(host(x)[0], ref.x) <= 2e-6
    s.close()


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("shape,nrhs", _random_shapes(3, 22))
def test_fixed_iteration_random_shapes(bc, shape, nrhs):
    """Five Bi-CGSTAB steps from x = 0 on seeded random shapes and right-hand
    sides, all right-hand sides in one batched solve: each iterate matches the
    oracle's single solve."""
    steps = 5
    h = 1.0 / (max(shape) - 1)
    k = hetero_k(shape, 23)
    lvl = Level(shape, h, k, bc)
    hier = build_hierarchy(k, h, bc)
    b = W.random_complex((nrhs,) + shape, seed=24) * unknown_mask(shape, bc)
    s = _solver(shape, h, bc, nrhs_max=nrhs)
    s.set_model(dev(k))
    s.set_sources(dev(b))
    x, st = s.solve(rtol=1e-14, maxit=steps)
    x = host(x)
    for i in range(nrhs):
        ref = O.bicgstab(lambda v: O.apply_A(v, lvl), lambda v: vcycle(v, hier), b[i], tol=1e-6,
                         fixed_iterations=steps)
        assert st[i].status == "HH_ERR_NOT_CONVERGED" and st[i].iterations == steps, (shape, i)
        assert relerr(x[i], ref.x) <= 1e-9, (shape, nrhs, i)
    s.close()


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("shape,nrhs", _random_shapes(3, 25))
def test_solve_random_shapes(bc, shape, nrhs):
    """Batched solves to relative residual 1e-6 on seeded random shapes (kh in
    [0.1, 0.4]), FP64 and mixed: every right-hand side stops with its true
    residual under the oracle's operator within the tolerance."""
    h = 1.0 / (max(shape) - 1)
    k = np.random.default_rng(26).uniform(0.1, 0.4, shape) / h
    lvl = Level(shape, h, k, bc)
    b = W.random_complex((nrhs,) + shape, seed=27) * unknown_mask(shape, bc)
    for prec in ("fp64", "mixed"):
        s = _solver(shape, h, bc, nrhs_max=nrhs, prec=prec)
        s.set_model(dev(k))
        s.set_sources(dev(b))
        x, st = s.solve(rtol=1e-6, maxit=500)
        x = host(x)
        for i in range(nrhs):
            assert st[i].status == "HH_OK", (shape, prec, i, st[i])
            true_rel = np.linalg.norm(b[i] - O.apply_A(x[i], lvl)) / np.linalg.norm(b[i])
            assert true_rel <= 1e-6, (shape, prec, i, true_rel)
        s.close()


def test_solve_wedge_small_mixed_and_fp64():
    """Down-scaled wedge (33 x 33 x 65), Sommerfeld: both precisions reach the
    true relative residual 1e-6 under the oracle's operator; the mixed solution
    is as close to the tight FP64 oracle solution as the FP64 one."""
    wl = W.wedge(10.0, 33, 33, 65)
    b = O.point_source_rhs(wl.shape, wl.h, wl.sources)[0]
    lvl = Level(wl.shape, wl.h, wl.k, wl.bc)
    tight, _ = _oracle_solve(wl, b, 1e-10)
    errs = {}
    for prec in ("fp64", "mixed"):
        s = _solver(wl.shape, wl.h, SOMMERFELD, prec=prec)
        s.set_model(dev(wl.k))
        s.set_point_sources(wl.sources)
        x, st = s.solve(rtol=1e-6)
        x = host(x)[0]
        rel = np.linalg.norm(b - O.apply_A(x, lvl)) / np.linalg.norm(b)
        assert st[0].status == "HH_OK" and rel <= 1e-6, (prec, rel)
        errs[prec] = np.linalg.norm(x - tight.x) / np.linalg.norm(tight.x)
    assert errs["mixed"] <= 10 * errs["fp64"] + 1e-7, errs


def test_batched_equals_single_solves_bitwise():
    wl = W.wedge(10.0, 17, 17, 33)
    nodes = [(0, 8, 8), (0, 3, 12), (0, 15, 1)]
    s = _solver(wl.shape, wl.h, SOMMERFELD, nrhs_max=4, prec="mixed")
    s.set_model(dev(wl.k))
    s.set_point_sources(nodes)
    xb, stb = s.solve(rtol=1e-8)
    xb = host(xb)
    for r, nd in enumerate(nodes):
        s.set_point_sources([nd])
        x1, st1 = s.solve(rtol=1e-8)
        assert np.array_equal(host(x1)[0], xb[r])
        assert st1[0].iterations == stb[r].iterations


def test_graph_and_direct_launch_bitwise_and_repeatable():
    wl = W.wedge(10.0, 17, 17, 33)
    s = _solver(wl.shape, wl.h, SOMMERFELD)
    s.set_model(dev(wl.k))
    s.set_point_sources(wl.sources)
    x1 = host(s.solve(rtol=1e-8)[0])
    x2 = host(s.solve(rtol=1e-8)[0])
    s.set_option("graph", 0)
    x3 = host(s.solve(rtol=1e-8)[0])
    s.set_option("graph", 1)
    s.set_option("check_every", 1)
    x4 = host(s.solve(rtol=1e-8)[0])
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3) and np.array_equal(x1, x4)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_traced_solve_bitwise_and_kernel_times(prec):
    """The event-traced solve runs the same kernels as the graph replay (same
    result bit for bit, also with the mixed form's restarts from x) and times
    every fine-level launch of the full windows (counted here without
    restarts, whose windows a right-hand side leaves early)."""
    wl = W.wedge(10.0, 17, 17, 33)
    nodes = [(0, 8, 8), (0, 4, 12)]
    s = _solver(wl.shape, wl.h, SOMMERFELD, prec=prec, nrhs_max=2)
    s.set_model(dev(wl.k))
    s.set_point_sources(nodes)
    for restart in ((1, 0) if prec == "mixed" else (0,)):
        s.set_option("restart_decade", restart)
        s.set_option("trace", 0)
        x1, st1 = s.solve(rtol=1e-8)
        x1 = host(x1)
        s.set_option("trace", 1)
        x2, st2 = s.solve(rtol=1e-8)
        x2 = host(x2)
        ms, n = s.kernel_times()
        s.set_option("trace", 0)
        assert np.array_equal(x1, x2), restart
        assert [a.iterations for a in st1] == [b.iterations for b in st2]
        assert [a.restarts for a in st1] == [b.restarts for b in st2]
        if restart:
            assert min(a.restarts for a in st1) >= 5
    # full windows: every right-hand side iterating; 4 steps per window
    steps = 4 * (int(min(a.iterations for a in st1)) // 4 - 1)
    assert steps > 0
    assert n[1] >= steps and n[4] == n[1] and n[5] == n[1] and n[6] == n[1]  # one launch per step
    assert n[0] == 2 * n[1] and n[2] == 2 * n[1] and n[3] == 2 * n[1]  # two per step
    assert all(0.0 < m < 50.0 for m in ms)
    assert ms[6] < ms[0]  # the empty bracket costs less than a working apply
    s.set_option("trace", 1)  # re-enabling resets the sums
    assert s.kernel_times()[1] == [0] * 7


def test_launch_shape_options_and_autotune():
    """Per-level z-block options, the stencil launch shape and the autotuner:
    every choice solves the same problem to the tolerance, and the multigrid
    result does not depend on the z-blocks (each node's arithmetic is fixed)."""
    from paper_2308_06085_amd._lib import HHError

    wl = W.wedge(10.0, 33, 33, 65)
    s = _solver(wl.shape, wl.h, SOMMERFELD, prec="mixed")
    s.set_model(dev(wl.k))
    s.set_point_sources(wl.sources)
    nlev = s.get_option("n_levels")
    first_tail = s.get_option("tail_first")
    assert 1 <= first_tail < nlev
    r = dev(W.random_complex(wl.shape, seed=3)).unsqueeze(0)
    z_ref = host(s.apply_vcycle(r))
    for zb in (1, 2, 3, 16):
        # every z-block of every level's passes gives the same bits
        for l in range(first_tail):
            for opt in (f"zb_down:{l}", f"zb_up:{l}"):
                s.set_option(opt, zb)
        assert np.array_equal(host(s.apply_vcycle(r)), z_ref), zb
    with pytest.raises(HHError):
        s.set_option(f"zb_down:{nlev - 1}", 2)   # the coarsest level has no pass
    with pytest.raises(HHError):
        s.set_option("zb_up:x", 2)
    for l in range(first_tail):
        s.set_option(f"zb_down:{l}", 0)
        s.set_option(f"zb_up:{l}", 0)
    for block, zb in ((128, 8), (512, 2)):
        s.set_option("block", block)
        s.set_option("zb", zb)
        x, st = s.solve(rtol=1e-7)
        assert st[0].status == "HH_OK" and st[0].relres_true <= 1e-7
    shapes = s.autotune()
    assert shapes["block"] in (128, 256, 512) and shapes["zb"] in (2, 4, 8)
    assert shapes["autotune_source"] == 2 and len(shapes["zb_down"]) == first_tail
    x, st = s.solve(rtol=1e-7)
    assert st[0].status == "HH_OK" and st[0].relres_true <= 1e-7
    # the tuned multigrid shapes leave the cycle's output unchanged bit for bit
    assert np.array_equal(host(s.apply_vcycle(r)), z_ref)


def test_resume_from_initial_guess():
    wl = W.wedge(10.0, 17, 17, 33)
    s = _solver(wl.shape, wl.h, SOMMERFELD)
    s.set_model(dev(wl.k))
    s.set_point_sources(wl.sources)
    x, st = s.solve(rtol=1e-8, maxit=2)
    assert st[0].status == "HH_ERR_NOT_CONVERGED"
    x2, st2 = s.solve(x0=x, rtol=1e-8)
    assert st2[0].status == "HH_OK" and st2[0].relres_true <= 1e-8


# --------------------------------------------------------------------------
# error behaviour
# --------------------------------------------------------------------------
def test_error_codes():
    from paper_2308_06085_amd._lib import HHError

    with pytest.raises(HHError) as e:
        _solver((9, 9, 8), 0.1, SOMMERFELD)
    assert e.value.status == 1
    s = _solver((9, 9, 9), 1 / 8, SOMMERFELD, nrhs_max=2)
    with pytest.raises(HHError) as e:
        s.set_point_sources([(4, 4, 4)])
        s.solve()
    assert e.value.status == 7  # no model yet
    k = np.full((9, 9, 9), 5.0)
    k[3, 3, 3] = np.nan
    with pytest.raises(HHError) as e:
        s.set_model(dev(k))
    assert e.value.status == 4
    s.set_model(dev(np.full((9, 9, 9), 5.0)))
    with pytest.raises(HHError) as e:
        s.set_point_sources([(4, 4, 4)] * 3)
    assert e.value.status == 1
    with pytest.raises(HHError) as e:
        s.set_point_sources([(4, 4, 9)])
    assert e.value.status == 1
    s.set_sources(torch.zeros((1, 9, 9, 9), dtype=torch.complex128, device="cuda"))
    x, st = s.solve(x0=torch.ones((1, 9, 9, 9), dtype=torch.complex128, device="cuda"))
    assert st[0].status == "HH_OK" and not host(x).any() and st[0].iterations == 0
    s.set_point_sources([(4, 4, 4)])
    x, st = s.solve(rtol=1e-14, maxit=1)
    assert st[0].status == "HH_ERR_NOT_CONVERGED" and st[0].iterations == 1
    d = _solver((9, 9, 9), 1 / 8, DIRICHLET)
    d.set_model(dev(np.full((9, 9, 9), 5.0)))
    with pytest.raises(HHError):
        d.set_point_sources([(0, 4, 4)])


def test_singular_dirichlet_operator_terminates():
    """k^2 on a discrete Dirichlet eigenvalue makes A singular: the solve must end
    with breakdown or non-convergence, never hang."""
    n = 9
    h = 1 / 8
    lam = 3 * 4 / h**2 * np.sin(np.pi * h / 2) ** 2
    s = _solver((n, n, n), h, DIRICHLET)
    s.set_model(dev(np.full((n, n, n), np.sqrt(lam))))
    s.set_point_sources([(4, 4, 4)])
    x, st = s.solve(rtol=1e-10, maxit=200)
    assert st[0].status in ("HH_OK", "HH_ERR_BREAKDOWN", "HH_ERR_NOT_CONVERGED", "HH_ERR_NUMERIC")


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------
def test_adjoint_kernels_match_oracle():
    from oracle.adjoint import adjoint_gradient_pointwise, adjoint_rhs

    shape = (9, 17, 13)
    rng = np.random.default_rng(12)
    s_sl = rng.uniform(1 / 3000**2, 1 / 1500**2, shape)
    u = W.random_complex((2,) + shape, 13)
    w = W.random_complex((2,) + shape, 14)
    g = W.random_complex((2,) + shape, 15)
    omega = 3000.0
    h = 0.1
    s = _solver(shape, h, SOMMERFELD, nrhs_max=2)
    s.set_model(dev(omega * np.sqrt(s_sl)))
    assert relerr(host(s.adjoint_rhs(dev(g))), adjoint_rhs(g, shape)) <= 1e-15
    grad = host(s.grad_slowness2(dev(u), dev(w), dev(s_sl), omega))
    ref = sum(adjoint_gradient_pointwise(u[r], w[r], s_sl, omega, h) for r in range(2))
    assert relerr(grad, ref) <= 1e-13


@pytest.mark.parametrize("shape,nrhs", _random_shapes(4, 34))
def test_adjoint_kernels_random_shapes(shape, nrhs):
    """The adjoint right-hand side and the pointwise gradient (summed over the
    right-hand sides) on seeded random shapes."""
    from oracle.adjoint import adjoint_gradient_pointwise, adjoint_rhs

    rng = np.random.default_rng(35)
    s_sl = rng.uniform(1 / 3000**2, 1 / 1500**2, shape)
    u = W.random_complex((nrhs,) + shape, 36)
    w = W.random_complex((nrhs,) + shape, 37)
    g = W.random_complex((nrhs,) + shape, 38)
    omega, h = 3000.0, 0.1
    s = _solver(shape, h, SOMMERFELD, nrhs_max=nrhs)
    s.set_model(dev(omega * np.sqrt(s_sl)))
    assert relerr(host(s.adjoint_rhs(dev(g))), adjoint_rhs(g, shape)) <= 1e-15, (shape, nrhs)
    grad = host(s.grad_slowness2(dev(u), dev(w), dev(s_sl), omega))
    ref = sum(adjoint_gradient_pointwise(u[r], w[r], s_sl, omega, h) for r in range(nrhs))
    assert relerr(grad, ref) <= 1e-13, (shape, nrhs)
    s.close()


def test_adjoint_gradient_autograd_vs_oracle_and_fd():
    """17^3 version of the adjoint workload through torch.autograd."""
    from oracle.adjoint import misfit_and_gradient, sample, solve_forward
    from paper_2308_06085_amd import HelmholtzSolve

    aw = W.adjoint_workload(17, ndir=6)
    b = O.point_source_rhs(aw.s_true.shape, aw.h, [aw.source])
    d = sample(solve_forward(aw.s_true, aw.omega, aw.h, b[0]).x, aw.receivers)
    s = _solver(aw.s_true.shape, aw.h, SOMMERFELD)
    rec = torch.tensor(aw.receivers, device="cuda")
    d_t = dev(d)

    def loss_fn(s_t):
        u = HelmholtzSolve.apply(s_t, dev(b), aw.omega, s, 1e-10)
        ur = u[0][rec[:, 0], rec[:, 1], rec[:, 2]]
        return 0.5 * torch.sum(torch.abs(ur - d_t) ** 2)

    s_t = dev(aw.s_model).requires_grad_(True)
    loss = loss_fn(s_t)
    loss.backward()
    g_gpu = host(s_t.grad)
    _, g_ref, _ = misfit_and_gradient(aw.s_model, aw.omega, aw.h, aw.source, aw.receivers, d)
    cos = float(np.sum(g_gpu * g_ref) / (np.linalg.norm(g_gpu) * np.linalg.norm(g_ref)))
    assert cos >= 0.9999, cos
    fd, ad = [], []
    with torch.no_grad():
        for v in aw.directions:
            lp = float(loss_fn(dev(aw.s_model + aw.eps * v)))
            lm = float(loss_fn(dev(aw.s_model - aw.eps * v)))
            fd.append((lp - lm) / (2 * aw.eps))
            ad.append(float(np.sum(g_gpu * v)))
    fd, ad = np.array(fd), np.array(ad)
    assert fd @ ad / (np.linalg.norm(fd) * np.linalg.norm(ad)) >= 0.999
