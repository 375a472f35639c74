"""The context-free, non-allocating operator apply (hh_apply_operator_noalloc)
against hh_apply_operator through the C ABI: two calls in a row on one device,
the second on a smaller grid, both boundary conditions; the arrays' values
must agree bit for bit (same kernel, same k^2), and match the oracle's A."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.discretization import Level

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _noalloc(lib, shape, h, bc, k, x):
    from paper_2308_06085_amd import _lib

    nz, ny, nx = shape
    cfg = _lib.Config()
    lib.hh_default_config(C.byref(cfg), nx, ny, nz, h)
    cfg.bc = _lib.BC[bc]
    y = torch.full_like(x, complex(np.nan, np.nan))
    st = lib.hh_apply_operator_noalloc(C.byref(cfg), k.data_ptr(), x.data_ptr(), y.data_ptr(), x.shape[0],
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.hh_last_error(None)
    return y


@pytest.mark.parametrize("bc", ["sommerfeld", "dirichlet"])
def test_noalloc_apply_equals_context_apply(bc):
    from paper_2308_06085_amd import Solver, _lib

    lib = _lib.load()
    # a larger grid with 3 right-hand sides, then a smaller one with 1: the
    # second call reuses the scratch the first one filled
    for shape, nrhs, seed in (((33, 65, 129), 3, 71), ((9, 17, 13), 1, 72)):
        h = 1.0 / (max(shape) - 1)
        k = np.random.default_rng(seed).uniform(4.0, 12.0, shape)
        x = W.random_complex((nrhs,) + shape, seed=seed + 100)
        kt, xt = dev(k), dev(x)
        s = Solver(shape, h, bc=bc, nrhs_max=nrhs)
        s.set_model(kt)
        y_ctx = host(s.apply_operator(xt))
        s.close()
        y = host(_noalloc(lib, shape, h, bc, kt, xt))
        assert np.array_equal(y, y_ctx), (shape, bc)
        ref = O.apply_A(x, Level(shape, h, k, bc))
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_noalloc_apply_binding_and_limits():
    from paper_2308_06085_amd import _lib
    from paper_2308_06085_amd.solver import apply_operator_noalloc

    shape = (17, 17, 33)
    h = 1.0 / 32
    k = dev(np.random.default_rng(73).uniform(4.0, 12.0, shape))
    x = dev(W.random_complex((2,) + shape, seed=74))
    y1 = host(apply_operator_noalloc(k, x, h))
    y2 = host(apply_operator_noalloc(k, x, h))
    assert np.array_equal(y1, y2)
    lib = _lib.load()
    cfg = _lib.Config()
    lib.hh_default_config(C.byref(cfg), 257, 257, 129, h)   # 8.5 M nodes > 2^23
    assert lib.hh_apply_operator_noalloc(C.byref(cfg), k.data_ptr(), x.data_ptr(), x.data_ptr(), 1, None) == 1
    assert b"no-allocation scratch" in lib.hh_last_error(None)
