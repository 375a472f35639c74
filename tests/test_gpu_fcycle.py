"""GPU parity of the F(1,1)-cycle preconditioner (paper section 3.4.5; option
"cycle" = 1) against the oracle's F-cycle, on the same seeded inputs.

Tolerances as for the V-cycle: one cycle in complex128 1e-12 relative to the
largest entry, complex64 1e-5 against the oracle's complex64 and complex128
cycles; fixed-iteration Bi-CGSTAB iterates 1e-9; iteration counts within
max(2, 5 %).  Shapes cover two to six levels and tails that start at levels
1 to 3, so the host recursion, the residual pass, the accumulating up pass and
both tail programs all run.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.discretization import DIRICHLET, SOMMERFELD, Level, unknown_mask
from oracle.multigrid import build_hierarchy, fcycle, vcycle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver(shape, h, bc, **kw):
    from paper_2308_06085_amd import Solver

    return Solver(shape, h, bc=bc, **kw)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def hetero_k(shape, seed, lo=4.0, hi=12.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


SHAPES = [(9, 9, 9), (5, 9, 65), (17, 9, 33), (33, 17, 17), (9, 65, 129), (33, 97, 41), (65, 33, 33)]


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("shape", SHAPES)
def test_fcycle_fp64(bc, shape):
    h = 1.0 / (max(shape) - 1)
    k = hetero_k(shape, 15)
    hier = build_hierarchy(k, h, bc)
    r = W.random_complex((2,) + shape, seed=16) * unknown_mask(shape, bc)
    s = _solver(shape, h, bc, nrhs_max=2, cycle="F")
    assert s.get_option("cycle") == 1
    assert s.level_shapes() == [lv.shape for lv in hier.levels]
    s.set_model(dev(k))
    z = host(s.apply_vcycle(dev(r)))
    ref = fcycle(r, hier)
    assert relerr(z, ref) <= 1e-12, (s.get_option("tail_first"), len(hier.levels))
    # switching back gives the V-cycle
    s.set_option("cycle", 0)
    assert relerr(host(s.apply_vcycle(dev(r))), vcycle(r, hier)) <= 1e-12


def _random_shapes(n, seed):
    """Seeded grid sizes m 2^j + 1 per axis (m = 1, 3, 5, 7: deep hierarchies
    with varying tails) with 1..4 right-hand sides."""
    sizes = [9, 13, 17, 21, 25, 29, 33, 41, 49, 57, 65]
    rng = np.random.default_rng(seed)
    return [(tuple(int(rng.choice(sizes)) for _ in range(3)), int(rng.integers(1, 5))) for _ in range(n)]


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("shape,nrhs", _random_shapes(4, 19))
def test_fcycle_random_shapes(bc, shape, nrhs):
    h = 1.0 / (max(shape) - 1)
    k = hetero_k(shape, 20)
    hier = build_hierarchy(k, h, bc)
    r = W.random_complex((nrhs,) + shape, seed=21) * unknown_mask(shape, bc)
    s = _solver(shape, h, bc, nrhs_max=nrhs, cycle="F")
    assert s.level_shapes() == [lv.shape for lv in hier.levels]
    s.set_model(dev(k))
    assert relerr(host(s.apply_vcycle(dev(r))), fcycle(r, hier)) <= 1e-12, (shape, nrhs)
    s.close()


def test_fcycle_wedge_deep_hierarchy():
    """65 x 65 x 129 wedge: six levels, tail from level 3, so the F-cycle's
    coarse-grid solve recurses through two fused levels before the tail; with
    beta2 = -1 (the shift the paper pairs with the F-cycle)."""
    wl = W.wedge(10.0, 65, 65, 129)
    for beta2 in (-0.5, -1.0):
        hier = build_hierarchy(wl.k, wl.h, wl.bc, beta2=beta2)
        s = _solver(wl.shape, wl.h, SOMMERFELD, cycle="F", beta=(1.0, beta2))
        s.set_model(dev(wl.k))
        assert s.get_option("n_levels") == 6 and s.get_option("tail_first") == 3
        r = W.random_complex(wl.shape, seed=17)
        z = host(s.apply_vcycle(dev(r)))[0]
        assert relerr(z, fcycle(r, hier)) <= 1e-12, beta2
        s.close()


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
def test_fcycle_mixed(bc):
    shape = (33, 33, 65)
    h = 1 / 64
    k = hetero_k(shape, 18)
    h64 = build_hierarchy(k, h, bc)
    h32 = build_hierarchy(k, h, bc, dtype=np.complex64)
    r = W.random_complex(shape, seed=19) * unknown_mask(shape, bc)
    s = _solver(shape, h, bc, prec="mixed", cycle="F")
    s.set_model(dev(k))
    z = host(s.apply_vcycle(dev(r)))[0]
    ref32 = fcycle(r.astype(np.complex64), h32).astype(np.complex128)
    ref64 = fcycle(r, h64)
    assert relerr(z, ref32) <= 1e-5
    assert relerr(z, ref64) <= 1e-5


def _oracle_fsolve(wl, b, tol, beta2=-0.5, **kw):
    lvl = Level(wl.shape, wl.h, wl.k, wl.bc)
    hier = build_hierarchy(wl.k, wl.h, wl.bc, beta2=beta2)
    return O.bicgstab(lambda x: O.apply_A(x, lvl), lambda r: fcycle(r, hier), b, tol=tol, **kw), lvl


@pytest.mark.parametrize("steps", [1, 3])
def test_fcycle_fixed_iteration_iterates(steps):
    shape = (17, 17, 33)
    h = 1 / 16
    k = hetero_k(shape, 20, 6.0, 14.0)
    wl = W.Workload(k, h, SOMMERFELD, [(8, 8, 16)], 0, "hetero")
    b = O.point_source_rhs(shape, h, wl.sources)[0]
    ref, _ = _oracle_fsolve(wl, b, 1e-6, fixed_iterations=steps)
    s = _solver(shape, h, SOMMERFELD, cycle="F")
    s.set_model(dev(k))
    s.set_point_sources(wl.sources)
    x, st = s.solve(rtol=1e-14, maxit=steps)
    assert st[0].status == "HH_ERR_NOT_CONVERGED" and st[0].iterations == steps
    assert relerr(host(x)[0], ref.x) <= 1e-9


@pytest.mark.parametrize("beta2", [-0.5, -1.0])
def test_fcycle_solve_wedge_small(beta2):
    """33 x 33 x 65 wedge: FP64 and mixed F-cycle solves reach the true relative
    residual 1e-6 under the oracle's operator, the FP64 iteration count matches
    the oracle's F-cycle Bi-CGSTAB, and at beta2 = -1 the F-cycle needs fewer
    iterations than the V-cycle (section 5's F-cycle experiments)."""
    wl = W.wedge(10.0, 33, 33, 65)
    b = O.point_source_rhs(wl.shape, wl.h, wl.sources)[0]
    ref, lvl = _oracle_fsolve(wl, b, 1e-6, beta2=beta2)
    its = {}
    for prec in ("fp64", "mixed"):
        for cyc in ("V", "F"):
            s = _solver(wl.shape, wl.h, SOMMERFELD, prec=prec, cycle=cyc, beta=(1.0, beta2))
            s.set_model(dev(wl.k))
            s.set_point_sources(wl.sources)
            x, st = s.solve(rtol=1e-6)
            x = host(x)[0]
            rel = np.linalg.norm(b - O.apply_A(x, lvl)) / np.linalg.norm(b)
            assert st[0].status == "HH_OK" and rel <= 1e-6, (prec, cyc, rel)
            its[prec, cyc] = st[0].iterations
            s.close()
    assert abs(its["fp64", "F"] - ref.iterations) <= max(2, 0.05 * ref.iterations), (its, ref.iterations)
    if beta2 == -1.0:
        assert its["fp64", "F"] < its["fp64", "V"], its


def test_fcycle_graph_batched_and_traced_bitwise():
    """Graph replay, direct launches and the event-traced solve give the same
    F-cycle result bit for bit; a batched right-hand side equals its single solve."""
    wl = W.wedge(10.0, 17, 17, 33)
    nodes = [(0, 8, 8), (0, 3, 12)]
    s = _solver(wl.shape, wl.h, SOMMERFELD, prec="mixed", cycle="F", nrhs_max=2)
    s.set_model(dev(wl.k))
    s.set_point_sources(nodes)
    xb, stb = s.solve(rtol=1e-8)
    xb = host(xb)
    s.set_option("graph", 0)
    assert np.array_equal(host(s.solve(rtol=1e-8)[0]), xb)
    s.set_option("graph", 1)
    s.set_option("trace", 1)
    assert np.array_equal(host(s.solve(rtol=1e-8)[0]), xb)
    s.set_option("trace", 0)
    s.set_point_sources([nodes[1]])
    x1, st1 = s.solve(rtol=1e-8)
    assert np.array_equal(host(x1)[0], xb[1]) and st1[0].iterations == stb[1].iterations


def test_cycle_option_errors():
    from paper_2308_06085_amd._lib import HHError

    s = _solver((9, 9, 9), 1 / 8, SOMMERFELD)
    with pytest.raises(HHError):
        s.set_option("cycle", 2)
    assert s.get_option("cycle") == 0
    with pytest.raises(ValueError):
        _solver((9, 9, 9), 1 / 8, SOMMERFELD, cycle="W")
