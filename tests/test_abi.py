"""The C-ABI library loads and exports every entry point include/hh.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hh.h")
LIB = os.path.join(ROOT, "paper_2308_06085_amd", "libhh.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hh_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hh_create", "hh_destroy", "hh_set_model", "hh_set_sources",
                     "hh_set_point_sources", "hh_solve", "hh_apply_operator",
                     "hh_apply_vcycle", "hh_adjoint_rhs", "hh_grad_slowness2"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libhh.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2308_06085_amd import _lib

    assert sorted(_lib.EXPORTS) == declared_functions()


def test_config_struct_layout_matches_header():
    """The ctypes mirror of hh_config / hh_stats has the C layout (field order and size)."""
    from paper_2308_06085_amd._lib import Config, Stats

    assert [f for f, _ in Config._fields_] == ["nx", "ny", "nz", "h", "bc", "beta1", "beta2",
                                               "omega", "nu_pre", "nu_post", "n_levels", "prec",
                                               "nrhs_max"]
    assert ctypes.sizeof(Config) == 80
    assert [f for f, _ in Stats._fields_] == ["iterations", "matvecs", "relres", "relres_true",
                                              "status", "restarts", "ms"]
    assert ctypes.sizeof(Stats) == 48


def test_default_config_and_create_validation_without_gpu():
    """hh_default_config and the argument checks of hh_create run on the host."""
    if not os.path.exists(LIB):
        pytest.skip("libhh.so not built")
    from paper_2308_06085_amd import _lib

    lib = _lib.load()
    cfg = _lib.Config()
    lib.hh_default_config(ctypes.byref(cfg), 33, 33, 65, 0.5)
    assert (cfg.nx, cfg.ny, cfg.nz, cfg.h) == (33, 33, 65, 0.5)
    assert (cfg.beta1, cfg.beta2, cfg.omega, cfg.bc) == (1.0, -0.5, 0.8, 1)
    assert (cfg.nu_pre, cfg.nu_post) == (1, 1)
    ctx = ctypes.c_void_p()
    for nu in ((2, 1), (1, 0), (0, 1)):
        # only one pre- and one post-smoothing sweep: rejected before any device call
        cfg.nu_pre, cfg.nu_post = nu
        assert lib.hh_create(ctypes.byref(cfg), None, ctypes.byref(ctx)) == 1
        assert b"nu_pre" in lib.hh_last_error(None)
    cfg.nu_pre = cfg.nu_post = 1
    cfg.nx = 32  # even: rejected before any device call
    assert lib.hh_create(ctypes.byref(cfg), None, ctypes.byref(ctx)) == 1
    assert b"odd" in lib.hh_last_error(None)


def test_create_rejects_planes_beyond_the_partial_sum_capacity():
    """An x-y plane whose operator-apply tiles alone exceed the reduction
    capacity is an argument error, found on the host before any device call."""
    if not os.path.exists(LIB):
        pytest.skip("libhh.so not built")
    from paper_2308_06085_amd import _lib

    lib = _lib.load()
    cfg = _lib.Config()
    lib.hh_default_config(ctypes.byref(cfg), 8193, 8193, 5, 1.0)
    ctx = ctypes.c_void_p()
    assert lib.hh_create(ctypes.byref(cfg), None, ctypes.byref(ctx)) == 1
    assert b"tiles" in lib.hh_last_error(None)


def test_noalloc_apply_validates_on_the_host():
    """The non-allocating apply rejects grids beyond its scratch and invalid
    arguments before any device call."""
    if not os.path.exists(LIB):
        pytest.skip("libhh.so not built")
    from paper_2308_06085_amd import _lib

    lib = _lib.load()
    cfg = _lib.Config()
    lib.hh_default_config(ctypes.byref(cfg), 257, 257, 129, 1.0)   # 8.5 M nodes > 2^23
    assert lib.hh_apply_operator_noalloc(ctypes.byref(cfg), 16, 16, 16, 1, None) == 1
    assert b"no-allocation scratch" in lib.hh_last_error(None)
    lib.hh_default_config(ctypes.byref(cfg), 9, 9, 9, 1.0)
    assert lib.hh_apply_operator_noalloc(ctypes.byref(cfg), 16, 16, 16, 0, None) == 1   # nrhs 0
    assert lib.hh_apply_operator_noalloc(ctypes.byref(cfg), None, 16, 16, 1, None) == 1  # null k
    cfg.ny = 8
    assert lib.hh_apply_operator_noalloc(ctypes.byref(cfg), 16, 16, 16, 1, None) == 1
