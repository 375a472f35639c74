"""The model given as squared slowness (hh_set_model_slowness2): the library's
k = omega sqrt(s) equals the same product formed on the host bit for bit, so
the operator and the cycle agree exactly with hh_set_model; invalid inputs are
errors; the autograd function sets the model once per forward/backward pair."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_slowness_model_equals_wavenumber_model(prec):
    from paper_2308_06085_amd import Solver

    n = 33
    h = 1.0 / (n - 1)
    c = W.smoothed_noise_velocity(n, seed=5)
    s2 = 1.0 / c**2
    omega = 0.5 * 1500.0 / h
    k = omega * np.sqrt(s2)
    x = dev(W.random_complex((1, n, n, n), seed=61))
    a = Solver((n, n, n), h, prec=prec)
    a.set_model(dev(k))
    b = Solver((n, n, n), h, prec=prec)
    b.set_model_slowness2(dev(s2), omega)
    assert np.array_equal(host(a.apply_operator(x)), host(b.apply_operator(x)))
    assert np.array_equal(host(a.apply_vcycle(x)), host(b.apply_vcycle(x)))
    a.close()
    b.close()


def test_slowness_model_errors():
    from paper_2308_06085_amd import Solver
    from paper_2308_06085_amd._lib import HHError

    n = 17
    s = Solver((n, n, n), 1.0 / (n - 1))
    s2 = np.full((n, n, n), 1.0 / 1500.0**2)
    with pytest.raises(HHError, match="HH_ERR_ARG"):
        s.set_model_slowness2(dev(s2), 0.0)
    bad = s2.copy()
    bad[3, 4, 5] = -1.0
    bad[0, 0, 0] = np.nan
    with pytest.raises(HHError, match="2 NaN/Inf or negative"):
        s.set_model_slowness2(dev(bad), 1000.0)
    # a failed set-up leaves no model: solving is out of order
    s.set_point_sources([(8, 8, 8)])
    with pytest.raises(HHError, match="HH_ERR_STATE"):
        s.solve()
    s.close()


def test_autograd_sets_the_model_once_per_gradient():
    from paper_2308_06085_amd import HelmholtzSolve, Solver

    n = 17
    h = 1.0 / (n - 1)
    s2 = dev(1.0 / W.smoothed_noise_velocity(n, seed=5) ** 2).requires_grad_(True)
    solver = Solver((n, n, n), h)
    b = torch.zeros((1, n, n, n), dtype=torch.complex128, device="cuda")
    b[0, 0, 8, 8] = 1.0 / h**3
    u = HelmholtzSolve.apply(s2, b, 0.4 * 1500.0 / h, solver, 1e-10)
    v0 = solver.model_version
    loss = 0.5 * torch.sum(torch.abs(u[0, 0]) ** 2)
    loss.backward()
    assert solver.model_version == v0     # backward reused the forward's model
    assert torch.isfinite(s2.grad).all() and float(torch.linalg.vector_norm(s2.grad)) > 0
    solver.close()
