"""Writes the oracle's Bi-CGSTAB step counts to relative residual 1e-6 on a
wedge problem (Sommerfeld), for 16 seeded top-face sources and the single
source at the centre of the top face, with the complex128 V-cycle (FP64),
with the complex64 V-cycle and shadow residual (mixed), and the same with
restarts from the current x at every power of ten of the residual
(mixed_restart, the library's default for the mixed form):

    wedge10      129 x 129 x 257 nodes, 10 Hz (kh up to 0.20)  -> wedge_step_counts.json
    halfwedge14   65 x  65 x 129 nodes, 14 Hz (kh up to 0.55)  -> half_wedge_14hz_step_counts.json

Bi-CGSTAB's step count on this indefinite problem reacts to roundings far
below the solution's accuracy: two preconditioners that differ by 1e-7 in
relative norm can need 10 % more or fewer steps on one source.  The mean over
many sources is what a change of precision actually moves, so the file keeps
every count and their means.  Calls only the oracle and the seeded input
generators; the 51 solves run in worker processes.

    python tests/golden/make_wedge_step_counts.py [wedge10|halfwedge14] [workers]
"""
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402
from oracle.discretization import Level  # noqa: E402
from oracle.multigrid import build_hierarchy, vcycle  # noqa: E402

N_SOURCES = 16
SOURCE_SEED = 4
RTOL = 1e-6
MAXIT = 1000
# name: (frequency in Hz, (nx, ny, nz), output file)
CONFIGS = {
    "wedge10": (10.0, (129, 129, 257), "wedge_step_counts.json"),
    "halfwedge14": (14.0, (65, 65, 129), "half_wedge_14hz_step_counts.json"),
}


def _workload(name):
    freq, (nx, ny, nz), _ = CONFIGS[name]
    return W.wedge(freq, nx, ny, nz)


def _count(job):
    name, prec, src = job
    wl = _workload(name)
    lvl = Level(wl.shape, wl.h, wl.k, wl.bc)
    if prec in ("mixed", "mixed_restart"):
        hier = build_hierarchy(wl.k, wl.h, wl.bc, n_levels=wl.n_levels, dtype=np.complex64)
        precond = lambda r: vcycle(r.astype(np.complex64), hier).astype(np.complex128)  # noqa: E731
        shadow = np.complex64
    else:
        hier = build_hierarchy(wl.k, wl.h, wl.bc, n_levels=wl.n_levels)
        precond = lambda r: vcycle(r, hier)  # noqa: E731
        shadow = None
    b = O.point_source_rhs(wl.shape, wl.h, [src])[0]
    res = O.bicgstab(lambda x: O.apply_A(x, lvl), precond, b, tol=RTOL, maxit=MAXIT, shadow_dtype=shadow,
                     restart_decade=prec == "mixed_restart")
    assert res.status == O.Status.OK and res.relres_true <= RTOL, (name, prec, src, res.status)
    return res.iterations


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "wedge10"
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else 4
    freq, (nx, ny, _), fname = CONFIGS[name]
    wl = _workload(name)
    sources = [tuple(int(v) for v in s)
               for s in W.batched_wedge_sources(N_SOURCES, seed=SOURCE_SEED, nx=nx, ny=ny)]
    single = tuple(int(v) for v in wl.sources[0])
    precs = ("mixed", "fp64", "mixed_restart")
    jobs = [(name, p, s) for p in precs for s in sources + [single]]
    t0 = time.time()
    with Pool(workers) as pool:
        counts = pool.map(_count, jobs, chunksize=1)
    out = {"problem": {"workload": "wedge", "freq": freq, "shape": list(wl.shape), "h": wl.h, "bc": wl.bc,
                       "rtol": RTOL, "sources": [list(s) for s in sources], "source_seed": SOURCE_SEED,
                       "single_source": list(single)},
           "seconds": round(time.time() - t0, 1)}
    n = len(sources) + 1
    for i, prec in enumerate(precs):
        c = counts[i * n:(i + 1) * n]
        out[prec] = {"steps": c[:-1], "mean": float(np.mean(c[:-1])), "single": c[-1]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), fname)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(path, {p: (out[p]["mean"], out[p]["single"]) for p in precs})


if __name__ == "__main__":
    main()
