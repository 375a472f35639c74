"""GPU parity of IDR(s) (paper section 3.1, the paper's IDR(4); option
"method" = 1) against the oracle's IDR(s) on the same seeded inputs and the
same shadow vectors.

The shadow vectors are drawn in complex64 (the library stores them in
complex64), so both sides use identical values.  Tolerances: fixed-step
iterates 1e-9 relative (complex128 throughout; summation order differs);
products-with-A counts of converged solves within max(3, 10 %) of the oracle's
(IDR(s), like Bi-CGSTAB, is sensitive to rounding); true relative residual
<= rtol under the oracle's operator.
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


def shadow64(s, shape, seed):
    """Shadow vectors with complex64-representable entries, as complex128."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((s,) + shape).astype(np.float32)
    im = rng.standard_normal((s,) + shape).astype(np.float32)
    return (re.astype(np.float64) + 1j * im.astype(np.float64)).astype(np.complex128)


def _hetero(shape, bc, seed):
    h = 1.0 / (max(shape) - 1)
    k = np.random.default_rng(seed).uniform(6.0, 14.0, shape)
    src = tuple(m // 2 for m in shape)
    return k, h, src


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("s,steps", [(4, 1), (4, 4), (4, 5), (4, 7), (4, 13), (1, 6), (2, 7), (8, 11)])
def test_idrs_fixed_step_iterates(bc, s, steps):
    shape = (17, 17, 33)
    k, h, src = _hetero(shape, bc, 31)
    lvl = Level(shape, h, k, bc)
    hier = build_hierarchy(k, h, bc)
    b = O.point_source_rhs(shape, h, [src])[0]
    P = shadow64(s, shape, 32)
    ref = O.idrs(lambda x: O.apply_A(x, lvl), lambda r: vcycle(r, hier), b, P, fixed_steps=steps)
    sv = _solver(shape, h, bc, method="idrs", idr_s=s)
    sv.set_model(dev(k))
    sv.set_shadow(dev(P))
    assert sv.get_option("idr_s") == s and sv.get_option("method") == 1
    sv.set_point_sources([src])
    x, st = sv.solve(rtol=1e-14, maxit=steps)
    assert st[0].status == "HH_ERR_NOT_CONVERGED" and st[0].iterations == steps, st[0]
    assert relerr(host(x)[0], ref.x) <= 1e-9


def _random_shapes(n, seed):
    """Seeded grid sizes m 2^j + 1 per axis (m = 1, 3, 5, 7: deep hierarchies)."""
    sizes = [9, 13, 17, 21, 25, 29, 33, 41, 49, 57, 65]
    rng = np.random.default_rng(seed)
    return [tuple(int(rng.choice(sizes)) for _ in range(3)) for _ in range(n)]


@pytest.mark.parametrize("bc", [SOMMERFELD, DIRICHLET])
@pytest.mark.parametrize("shape", _random_shapes(3, 36))
def test_idrs_fixed_step_random_shapes(bc, shape):
    """Six IDR(4) products on seeded random shapes with a random right-hand side."""
    steps = 6
    h = 1.0 / (max(shape) - 1)
    k = np.random.default_rng(37).uniform(6.0, 14.0, shape)
    lvl = Level(shape, h, k, bc)
    hier = build_hierarchy(k, h, bc)
    b = W.random_complex(shape, seed=38) * unknown_mask(shape, bc)
    P = shadow64(4, shape, 39)
    ref = O.idrs(lambda x: O.apply_A(x, lvl), lambda r: vcycle(r, hier), b, P, fixed_steps=steps)
    sv = _solver(shape, h, bc, method="idrs", idr_s=4)
    sv.set_model(dev(k))
    sv.set_shadow(dev(P))
    sv.set_sources(dev(b))
    x, st = sv.solve(rtol=1e-14, maxit=steps)
    assert st[0].status == "HH_ERR_NOT_CONVERGED" and st[0].iterations == steps, (shape, st[0])
    assert relerr(host(x)[0], ref.x) <= 1e-9, shape
    sv.close()


@pytest.mark.parametrize("steps", [3, 7])
def test_idrs_fcycle_fixed_step_iterates(steps):
    """IDR(4) with the F(1,1)-cycle preconditioner (the paper's F-cycle runs of
    section 5) against the oracle's idrs with its fcycle."""
    shape = (17, 17, 33)
    k, h, src = _hetero(shape, SOMMERFELD, 34)
    lvl = Level(shape, h, k, SOMMERFELD)
    hier = build_hierarchy(k, h, SOMMERFELD, beta2=-1.0)
    b = O.point_source_rhs(shape, h, [src])[0]
    P = shadow64(4, shape, 35)
    ref = O.idrs(lambda x: O.apply_A(x, lvl), lambda r: fcycle(r, hier), b, P, fixed_steps=steps)
    sv = _solver(shape, h, SOMMERFELD, method="idrs", idr_s=4, cycle="F", beta=(1.0, -1.0))
    sv.set_model(dev(k))
    sv.set_shadow(dev(P))
    sv.set_point_sources([src])
    x, st = sv.solve(rtol=1e-14, maxit=steps)
    assert st[0].status == "HH_ERR_NOT_CONVERGED" and st[0].iterations == steps, st[0]
    assert relerr(host(x)[0], ref.x) <= 1e-9


def test_idr1_with_r0_shadow_equals_bicgstab_on_gpu():
    """IDR(1) with the shadow vector b (= r_0 from x_0 = 0) and kappa = 0 is
    Bi-CGSTAB: after 2j products its iterate is the GPU Bi-CGSTAB's after j steps."""
    shape = (17, 17, 33)
    k, h, src = _hetero(shape, SOMMERFELD, 33)
    b = O.point_source_rhs(shape, h, [src])
    bi = _solver(shape, h, SOMMERFELD)
    bi.set_model(dev(k))
    bi.set_point_sources([src])
    idr = _solver(shape, h, SOMMERFELD, method="idrs", idr_s=1)
    idr.set_model(dev(k))
    idr.set_point_sources([src])
    idr.set_shadow(dev(b))  # 1/h^3 at one node: exact in complex64
    idr.set_option("idr_kappa_milli", 0)
    for j in (1, 3):
        xb, _ = bi.solve(rtol=1e-14, maxit=j)
        xi, _ = idr.solve(rtol=1e-14, maxit=2 * j)
        assert relerr(host(xi)[0], host(xb)[0]) <= 1e-10, j


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_idrs_solve_wedge_small(prec):
    """33 x 33 x 65 wedge, IDR(4): true relative residual <= 1e-6 under the
    oracle's operator; FP64 products-with-A count close to the oracle's."""
    wl = W.wedge(10.0, 33, 33, 65)
    lvl = Level(wl.shape, wl.h, wl.k, wl.bc)
    b = O.point_source_rhs(wl.shape, wl.h, wl.sources)[0]
    P = shadow64(4, wl.shape, 34)
    s = _solver(wl.shape, wl.h, SOMMERFELD, prec=prec, method="idrs")
    s.set_model(dev(wl.k))
    s.set_shadow(dev(P))
    s.set_point_sources(wl.sources)
    x, st = s.solve(rtol=1e-6)
    x = host(x)[0]
    rel = np.linalg.norm(b - O.apply_A(x, lvl)) / np.linalg.norm(b)
    assert st[0].status == "HH_OK" and rel <= 1e-6, (rel, st[0])
    assert abs(st[0].relres_true - rel) <= 1e-9
    if prec == "fp64":
        hier = build_hierarchy(wl.k, wl.h, wl.bc)
        ref = O.idrs(lambda v: O.apply_A(v, lvl), lambda r: vcycle(r, hier), b, P)
        assert abs(st[0].iterations - ref.iterations) <= max(3, 0.1 * ref.iterations), (st[0], ref.iterations)
        assert st[0].matvecs == st[0].iterations + 1 + st[0].restarts


def test_idrs_closed_off_dirichlet_against_oracle():
    """Closed-off problem (section 2.1), 33^3, k = 20, Dirichlet: the GPU IDR(4)
    solution reaches 1e-6, its products-with-A count is the oracle's within
    max(3, 10 %) with the same shadow vectors, and it is as close to a tight
    oracle solution as a 1e-6 solve can be (its distance to the analytic
    solution is the grid's discretisation error, 1.1e-2 at kh = 0.625)."""
    lvl, b, uex = O.closed_off_problem(33, 20.0)
    hier = build_hierarchy(lvl.k, lvl.h, lvl.bc)
    P = shadow64(4, lvl.shape, 35) * unknown_mask(lvl.shape, DIRICHLET)
    ref = O.idrs(lambda v: O.apply_A(v, lvl), lambda r: vcycle(r, hier), b, P)
    s = _solver(lvl.shape, lvl.h, DIRICHLET, method="idrs")
    s.set_model(dev(lvl.k))
    s.set_shadow(dev(P))
    s.set_sources(dev(b))
    x, st = s.solve(rtol=1e-6)
    x = host(x)[0]
    rel = np.linalg.norm(b - O.apply_A(x, lvl)) / np.linalg.norm(b)
    assert st[0].status == "HH_OK" and rel <= 1e-6
    assert abs(st[0].iterations - ref.iterations) <= max(3, 0.1 * ref.iterations), (st[0], ref.iterations)
    tight = O.idrs(lambda v: O.apply_A(v, lvl), lambda r: vcycle(r, hier), b, P, tol=1e-12)
    assert np.linalg.norm(x - tight.x) <= 1e-4 * np.linalg.norm(tight.x)
    assert abs(np.abs(x - uex).max() - np.abs(tight.x - uex).max()) <= 1e-4


def test_idrs_batched_graph_and_generated_shadow():
    """Batched right-hand sides equal their single solves bit for bit; graph
    replay equals direct launches; the generated shadow vectors converge and
    are repeatable; option and argument errors."""
    from paper_2308_06085_amd._lib import HHError

    wl = W.wedge(10.0, 17, 17, 33)
    nodes = [(0, 8, 8), (0, 3, 12)]
    s = _solver(wl.shape, wl.h, SOMMERFELD, prec="mixed", method="idrs", nrhs_max=2)
    s.set_model(dev(wl.k))
    s.set_point_sources(nodes)
    xb, stb = s.solve(rtol=1e-8)
    xb = host(xb)
    assert all(t.status == "HH_OK" for t in stb)
    s.set_option("graph", 0)
    assert np.array_equal(host(s.solve(rtol=1e-8)[0]), xb)
    s.set_option("graph", 1)
    s.set_point_sources([nodes[1]])
    x1, st1 = s.solve(rtol=1e-8)
    assert np.array_equal(host(x1)[0], xb[1]) and st1[0].iterations == stb[1].iterations
    s.set_option("idr_seed", 7)
    x7, st7 = s.solve(rtol=1e-8)
    assert st7[0].status == "HH_OK" and not np.array_equal(host(x7)[0], xb[1])
    with pytest.raises(HHError):
        s.set_option("idr_s", 9)
    with pytest.raises(HHError):
        s.set_option("method", 3)
    with pytest.raises(HHError):
        s.set_shadow(dev(np.zeros((9,) + wl.shape, dtype=np.complex128)))
    # back to Bi-CGSTAB on the same context
    s.set_option("method", 0)
    xbi, stbi = s.solve(rtol=1e-8)
    assert stbi[0].status == "HH_OK"


def test_idrs_shadow_dimension_change_on_one_context():
    """Growing s on a context that has already solved (new buffers, new captured
    cycles) gives the result of a fresh context with that s, bit for bit."""
    wl = W.wedge(10.0, 17, 17, 33)
    P2, P8 = shadow64(2, wl.shape, 51), shadow64(8, wl.shape, 52)

    def make():
        s = _solver(wl.shape, wl.h, SOMMERFELD, method="idrs")
        s.set_model(dev(wl.k))
        s.set_point_sources(wl.sources)
        return s

    a = make()
    a.set_shadow(dev(P2))
    xa2, sta2 = a.solve(rtol=1e-8)
    a.set_shadow(dev(P8))
    assert a.get_option("idr_s") == 8
    xa8, sta8 = a.solve(rtol=1e-8)
    b = make()
    b.set_shadow(dev(P8))
    xb8, stb8 = b.solve(rtol=1e-8)
    assert sta2[0].status == "HH_OK" and sta8[0].status == "HH_OK"
    assert np.array_equal(host(xa8), host(xb8)) and sta8[0].iterations == stb8[0].iterations
