"""The autotuner's cache file and its shapes: the per-level multigrid z-blocks
and down-pass regions it picks leave the cycle's output unchanged bit for bit,
tuned solves meet the tolerance, a cached entry is applied without measuring,
and a malformed cache file is an argument error."""
import json

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


def _solver(wl, **kw):
    from paper_2308_06085_amd import Solver

    return Solver(wl.shape, wl.h, bc=wl.bc, n_levels=wl.n_levels, **kw)


@pytest.mark.parametrize("prec,nrhs", [("mixed", 3), ("fp64", 1)])
def test_autotune_cache_roundtrip(tmp_path, prec, nrhs):
    wl = W.wedge(10.0, 33, 33, 65)
    nodes = W.batched_wedge_sources(nrhs, seed=4, nx=33, ny=33)
    cache = tmp_path / "tune.json"
    r = dev(W.random_complex((nrhs,) + wl.shape, seed=51))

    s = _solver(wl, prec=prec, nrhs_max=nrhs)
    s.set_model(dev(wl.k))
    s.set_point_sources(nodes)
    z_default = host(s.apply_vcycle(r))
    assert s.get_option("autotune_source") == 0
    tuned = s.autotune(cache)
    assert tuned["autotune_source"] == 2
    levels = s.get_option("tail_first")
    assert len(tuned["zb_down"]) == len(tuned["zb_up"]) == len(tuned["dn_region"]) == levels
    assert all(z in (1, 2, 4, 8, 16) for z in tuned["zb_down"] + tuned["zb_up"])
    assert all(g in (256, 512, 1280) for g in tuned["dn_region"])
    # the tuned multigrid shapes change no bit of the cycle
    assert np.array_equal(host(s.apply_vcycle(r)), z_default)
    x, st = s.solve(rtol=1e-7)
    assert all(t.status == "HH_OK" and t.relres_true <= 1e-7 for t in st), st
    assert all(t.ms > 0 for t in st)

    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    key, entry = next(iter(entries.items()))
    assert f"|33x33x65|sommerfeld|{prec}|nrhs{nrhs}|V|levels" in key
    assert entry["block"] == tuned["block"] and entry["zb"] == tuned["zb"]
    assert entry["zb_down"] == [s.get_option(f"zb_down:{l}") for l in range(levels)]
    assert entry["step_ms"] > 0 and entry["default_step_ms"] > 0
    s.close()

    # a second context with the same key takes the entry without measuring
    s2 = _solver(wl, prec=prec, nrhs_max=nrhs)
    s2.set_model(dev(wl.k))
    s2.set_point_sources(nodes)
    got = s2.autotune(cache)
    assert got["autotune_source"] == 1
    for f in ("block", "zb", "zb_down", "zb_up"):
        assert got[f] == tuned[f], f
    assert np.array_equal(host(s2.apply_vcycle(r)), z_default)
    x2, st2 = s2.solve(rtol=1e-7)
    # same shapes, same rounding: the solves agree bit for bit
    assert np.array_equal(host(x2), host(x)) and [t.iterations for t in st2] == [t.iterations for t in st]
    s2.close()


def test_autotune_cache_errors(tmp_path):
    from paper_2308_06085_amd._lib import HHError

    wl = W.wedge(10.0, 17, 17, 33)
    s = _solver(wl)
    s.set_model(dev(wl.k))
    with pytest.raises(HHError):
        s.autotune()          # no sources set
    s.set_point_sources(wl.sources)
    bad = tmp_path / "bad.json"
    bad.write_text("[1, 2, 3]")
    with pytest.raises(HHError, match="not a JSON object"):
        s.autotune(bad)
    assert bad.read_text() == "[1, 2, 3]"   # left as it was
    # an entry for this key with a shape outside the tuned sets
    good = tmp_path / "tune.json"
    s.autotune(good)
    entries = json.loads(good.read_text())
    key = next(iter(entries))
    entries[key]["zb_up"][0] = 3
    good.write_text(json.dumps(entries))
    with pytest.raises(HHError, match="outside"):
        s.autotune(good)
    s.close()
