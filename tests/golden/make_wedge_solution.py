"""Writes wedge_solution_samples.json: the oracle's solution of the wedge
problem (129 x 129 x 257 nodes, 10 Hz, Sommerfeld, point source at the centre
of the top face) solved to relative residual 1e-10 by its Bi-CGSTAB with the
complex128 V-cycle, at a seeded sample of nodes, with the solution's 2-norm
and largest modulus.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_wedge_solution.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402
from oracle.discretization import Level  # noqa: E402
from oracle.multigrid import build_hierarchy, vcycle  # noqa: E402

N_SAMPLES = 2048
SEED = 71


def main():
    wl = W.wedge(10.0)
    lvl = Level(wl.shape, wl.h, wl.k, wl.bc)
    hier = build_hierarchy(wl.k, wl.h, wl.bc, n_levels=wl.n_levels)
    b = O.point_source_rhs(wl.shape, wl.h, wl.sources)[0]
    t0 = time.time()
    res = O.bicgstab(lambda x: O.apply_A(x, lvl), lambda r: vcycle(r, hier), b, tol=1e-10)
    assert res.status == O.Status.OK and res.relres_true <= 1e-10, res.status
    x = res.x.ravel()
    rng = np.random.default_rng(SEED)
    idx = np.sort(rng.choice(x.size, size=N_SAMPLES, replace=False))
    # the source node and its neighbourhood, where the solution is largest
    sz, sy, sx = wl.sources[0]
    nz, ny, nx = wl.shape
    near = [(sz + dz) * ny * nx + (sy + dy) * nx + (sx + dx)
            for dz in (0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    idx = np.unique(np.concatenate([idx, np.array(near)]))
    out = {
        "problem": {"workload": "wedge", "freq": 10.0, "shape": list(wl.shape), "h": wl.h, "bc": wl.bc,
                    "source": list(wl.sources[0]), "tol": 1e-10, "preconditioner": "complex128 V-cycle"},
        "oracle": {"iterations": res.iterations, "relres_true": res.relres_true,
                   "seconds": round(time.time() - t0, 1)},
        "norm2": float(np.linalg.norm(x)),
        "max_abs": float(np.abs(x).max()),
        "index": [int(i) for i in idx],
        "re": [float(v) for v in x[idx].real],
        "im": [float(v) for v in x[idx].imag],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wedge_solution_samples.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(path, out["oracle"])


if __name__ == "__main__":
    main()
