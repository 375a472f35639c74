"""Benchmark: DoF-iterations/s of CSLP-preconditioned Bi-CGSTAB on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
                    [--workload cube513|wedge|batched|beta2_sweep|closedoff129]

One step = one complete solve to ||b - A x|| / ||b|| <= 1e-6 of the workload
(model and sources resident in HBM before the timed region).  The default
workload is the constant-k unit cube on 513^3 nodes (135,005,697 unknowns,
h = 1/512, k = 160 so kh = 0.3125, first-order Sommerfeld boundaries, 8
multigrid levels down to 5^3, one point source at the centre node): at 2.16 GB
per complex128 vector nothing of a step stays in the 256 MB Infinity Cache.
``value`` is the mixed-precision solve (complex64 V-cycle inside complex128
Bi-CGSTAB), K timed solves after W warm-up solves; the plain complex128 solve
is timed the same way (on the cube at most 5 timed solves after at most one
warm-up: its step count is deterministic) and reported under ``fp64``.

DoF-iterations/s = unknowns x Bi-CGSTAB iterations (half step = 0.5, summed
over right-hand sides) / solve time.

``roofline`` reports the kernel with the largest share of an iteration.  After
the timed solves a few more solves of the same workload (2 on the cube, else K)
run with the library's event tracing on: HIP events on the solver's stream
around every fine-level launch of every step (the steps launched directly
instead of replayed as a graph; only check windows in which every right-hand
side kept iterating count).  ``avg_ms`` is the kernel's average event-bracketed
duration over those launches (``launches`` of them), nothing subtracted, so it
is comparable with the per-dispatch mean of a rocprofv3 kernel trace of the
same command; ``event_bracket_ms`` (events around one launch whose workgroups
all exit at once) is reported beside it as the bracket's own cost.
``achieved`` = the kernel's algorithmic bytes per launch / ``avg_ms``, against
8 TB/s HBM3E peak.
``hbm_per_iteration``: the algorithmic bytes of one whole Bi-CGSTAB step as
built (every kernel of KERNELS, the coarse multigrid levels at 1/7 of the
level-0 passes) per DoF, times DoF x iterations / solve time: the whole
iteration's HBM rate, beside the dominant kernel's.
``cpu_baseline`` times the CPU oracle on a bounded sample of the workload on
the host (NumPy, BLAS held to one thread), set-up excluded: one complex128
Bi-CGSTAB step of the 513^3 cube itself (8 steps of the wedge).  If the host
lacks the free memory (about 400 B per node), the sample is the largest
2^j + 1 cube with the same kh that fits, and ``sample`` says so.

``variants`` (wedge workload): the same solves with the paper's other
solver settings, both precisions, timed the same way: Bi-CGSTAB with one
F(1,1)-cycle (section 3.4.5), IDR(4) (section 3.1) with the V- and with the
F-cycle, and full GMRES (left preconditioning, stopped on the preconditioned
residual as in the paper) with the V- and the F-cycle.  Each gives iterations
(Bi-CGSTAB steps, IDR products with A, GMRES Arnoldi steps), products with A
(``matvecs``, the paper's #Matvec), time per solve, the true relative
residual, and the time-to-solution ratio against the headline Bi-CGSTAB +
V-cycle solve.  The batched workload reports Bi-CGSTAB with the F-cycle.

``--method idrs`` / ``--cycle F`` change the headline solves themselves.

``--workload beta2_sweep``: the paper's F-cycle experiment (section 5), the
wedge at 40 Hz on 193 x 193 x 321 nodes (h = 3.125 m), mixed precision,
Bi-CGSTAB, IDR(4) and GMRES, V- and F-cycle, for beta2 = -0.5 ... -1.0:
iterations, products with A and time per solve to 1e-6 (at most 1200
products with A, 400 GMRES steps); ``value`` is the fastest solve's time in ms.

``--workload closedoff129``: the closed-off problem of section 2.1 on 129^3
nodes with k = 40 and the coarsening stopped at 17^3 (the configuration of the
paper's scaling runs, section 5.2): GMRES, IDR(4) and Bi-CGSTAB with the
V-cycle, FP64 and mixed, to relative residual 1e-6; ``value`` is the FP64
IDR(4) solve's time in ms, every run is listed under ``runs``.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DoF-iterations/s of CSLP-Bi-CGSTAB, mixed vs FP64 at 1e-6 rel residual; %HBM"

# Kernel ids of hh_time_kernel, launches per Bi-CGSTAB step and algorithmic
# bytes per fine-grid node for (fp64, mixed) precision: every array the kernel
# must read or write once (complex128 16 B, complex64 8 B, real k^2 8 B for the
# operator, k in the multigrid precision for the multigrid passes, coarse-grid
# arrays 1/8 of a fine one), split into the bytes of each right-hand side and
# the bytes all right-hand sides of a batch share (k^2, k: read once per launch).  In the mixed solve
# the preconditioner's inputs (complex64 copies of p and s, written by the p
# and s updates), its outputs p_hat, s_hat and the shadow residual r_hat are
# complex64.  The operator apply's figure is the mean of its two launches per
# step: v = A p_hat with r_hat^H v (FP64 56 B, mixed 40 B) and t = A s_hat with
# t^H s, t^H t (FP64 56 B, mixed 48 B: s stays complex128).  The x / r update
# alternates: an even step reads s, t, r_hat and writes r (FP64 64 B, mixed
# 56 B); an odd step also reads x and both steps' p_hat, s_hat and writes x
# (FP64 160 B, mixed 120 B); its figure is the mean of the two.
KERNELS = {  # id: (name, launches per step, per-RHS (fp64, mixed), shared (fp64, mixed))
    0: ("apply_A+dots", 2, (16 + 16 + 16, 8 + (8 + 16) / 2 + 16), (8, 8)),
    1: ("update_xr+dots", 1, ((64 + 160) / 2, (56 + 120) / 2), (0, 0)),
    2: ("mg_down_L0", 2, (16 + 16 / 8, 8 + 8 / 8), (8, 4)),
    3: ("mg_up_L0", 2, (16 + 16 / 8 + 16, 8 + 8 / 8 + 8), (8, 4)),
    4: ("p_update", 1, (4 * 16, 4 * 16 + 8), (0, 0)),
    5: ("s_update+dot", 1, (3 * 16, 3 * 16 + 8), (0, 0)),
}


def kernel_bytes(kid: int, prec_idx: int, nrhs: int = 1) -> float:
    """Algorithmic bytes per fine node of one launch of kernel `kid` for
    `nrhs` right-hand sides."""
    _, _, rhs, shared = KERNELS[kid]
    return nrhs * rhs[prec_idx] + shared[prec_idx]


# Coarse multigrid levels per preconditioner application: the level-0 pass
# bytes (down + up) times sum_{l>=1} 8^-l = 1/7; two applications per step.
def step_bytes(prec_idx: int, nrhs: int = 1) -> float:
    """Algorithmic bytes per fine node of one Bi-CGSTAB step for `nrhs`
    iterating right-hand sides as built: every level-0 kernel of KERNELS times
    its launches per step, plus the coarse levels."""
    total = sum(KERNELS[k][1] * kernel_bytes(k, prec_idx, nrhs) for k in KERNELS)
    mg = kernel_bytes(2, prec_idx, nrhs) + kernel_bytes(3, prec_idx, nrhs)
    return total + 2 * mg / 7.0


def step_bytes_per_dof(prec_idx: int) -> float:
    """Algorithmic bytes per DoF of one single-source Bi-CGSTAB step."""
    return step_bytes(prec_idx, 1)


# HBM traffic per launch, FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (scale factors
# from a 1 GiB reference copy; the operator apply's entry is the mean of its two
# launches in a step, the x / r update's the mean of its even- and odd-step
# launches) from two rocprofv3 --pmc runs of
# `bench.py --steps 1 --warmup 0 --no-cpu --no-fp64 --copy-calibration`
# (profiles/cube513_hbm_traffic.md).  Valid only for the kernel sources it was
# measured on (kernel_source_sha); otherwise reported as null.
TRAFFIC = {
    ("update_xr+dots", "cube513", "mixed"): (11886.4e6, "bdf21719b2142df3"),
    ("apply_A+dots", "cube513", "mixed"): (6241.9e6, "bdf21719b2142df3"),
    ("mg_down_L0", "cube513", "mixed"): (2313.0e6, "bdf21719b2142df3"),
    ("mg_up_L0", "cube513", "mixed"): (3226.4e6, "bdf21719b2142df3"),
    ("p_update", "cube513", "mixed"): (9720.4e6, "bdf21719b2142df3"),
    ("s_update+dot", "cube513", "mixed"): (7562.3e6, "bdf21719b2142df3"),
}


# the sources that define the kernels of the TRAFFIC table (the operator apply
# and Krylov updates, the multigrid passes) and the device headers they include
TRAFFIC_SOURCES = ("hh_kernels.hip", "hh_mg_fused.hip", "hh_common.h", "hh_device.h", "hh_kernels.h")


def kernel_source_sha() -> str:
    """sha256 (16 hex digits) of the code of the kernels in TRAFFIC: their
    sources with `//` comments and blank lines left out, so that a change to
    a comment keeps the counters and any change to the code drops them."""
    import re

    csrc = os.path.join(ROOT, "paper_2308_06085_amd", "csrc")
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"//[^\"]*$", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def streaming_reference(torch) -> dict:
    """The rate of PyTorch's own streaming kernels on this device, as a practical
    HBM ceiling beside the 8 TB/s peak: c = a + b (two reads, one write) and a
    copy, on 2 GiB float64 vectors, 20 launches each timed with HIP events."""
    n = (2 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)

    def rate(fn, nbytes, reps=20):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9

    add = rate(lambda: torch.add(a, b, out=c), 3 * 8 * n)
    copy = rate(lambda: c.copy_(a), 2 * 8 * n)
    del a, b, c
    torch.cuda.empty_cache()
    return {"kernel": "torch.add c = a + b on 2 GiB float64 vectors (2 reads + 1 write)",
            "GBs": round(add, 1), "copy_GBs": round(copy, 1)}


def closed_off_runs(args, n=129, kk=40.0):
    """The paper's closed-off problem (section 2.1; its scaling runs of section
    5.2) on n^3 nodes with k = 40 and the coarsening stopped at 17^3: GMRES,
    IDR(4) and Bi-CGSTAB with the V-cycle, FP64 and mixed, to relative residual
    1e-6 (the preconditioned one for GMRES)."""
    import torch

    import workloads as W
    from paper_2308_06085_amd import Solver

    k, b, _ = W.closed_off_rhs(n, kk)
    k, b = torch.from_numpy(k).cuda(), torch.from_numpy(b).cuda()
    levels = int(round(math.log2((n - 1) / 16))) + 1
    unknowns = (n - 2) ** 3
    rows = []
    for prec in ("fp64", "mixed"):
        for method in ("gmres", "idrs", "bicgstab"):
            s = Solver((n, n, n), 1.0 / (n - 1), bc="dirichlet", prec=prec, n_levels=levels, method=method)
            assert s.level_shapes()[-1] == (17, 17, 17)
            s.set_model(k)
            s.set_sources(b)
            warm, reps = (0, 1) if method == "gmres" else (args.warmup, args.steps)
            x = None
            for _ in range(warm):
                x, _ = s.solve(rtol=1e-6, maxit=2000, out=x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                x, st = s.solve(rtol=1e-6, maxit=2000, out=x)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
            rows.append({"precision": prec, "method": method, "iterations": st[0].iterations,
                         "matvecs": st[0].matvecs, "status": st[0].status, "relres": st[0].relres,
                         "relres_true": st[0].relres_true, "ms_per_solve": ms,
                         "dof_matvecs_per_s": unknowns * st[0].matvecs / (ms * 1e-3)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            s.close()
            del x
    head = next(r for r in rows if r["precision"] == "fp64" and r["method"] == "idrs")
    line = {
        "metric": "time to 1e-6 rel residual, closed-off problem with a 17^3 coarsest grid: GMRES, IDR(4), Bi-CGSTAB",
        "value": head["ms_per_solve"], "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128 (fp64 rows) / c64 cycle + c128 Krylov (mixed rows)", "data": "synthetic",
        "config": {"workload": f"closed-off {n}^3 k={kk:g} Dirichlet u=1, {levels} levels down to 17^3",
                   "unknowns": unknowns, "nrhs": 1, "rtol": 1e-6, "headline_row": "fp64 IDR(4)"},
        "runs": rows,
    }
    print(json.dumps(line), flush=True)


def make_workload(name):
    import workloads as W

    if name == "wedge":
        wl = W.wedge(10.0)
        return wl, wl.sources, "wedge 129x129x257 f=10Hz h=4.6875m Sommerfeld, 1 source"
    if name == "cube513":
        wl = W.big_cube()
        return wl, wl.sources, "cube 513^3 k=160 kh=0.3125 Sommerfeld, 8 levels, 1 source"
    if name == "beta2_sweep":
        wl = W.wedge(40.0, 193, 193, 321)
        return wl, wl.sources, "wedge 193x193x321 f=40Hz h=3.125m Sommerfeld, 1 source"
    if name == "batched":
        wl = W.wedge(10.0)
        src = W.batched_wedge_sources(16, seed=4)
        return wl, src, "wedge 129x129x257 f=10Hz, 16 seeded top-face sources, one batched solve"
    raise SystemExit(f"unknown workload {name}")


def dof(wl):
    nz, ny, nx = wl.shape
    if wl.bc == "sommerfeld":
        return nz * ny * nx
    return (nz - 2) * (ny - 2) * (nx - 2)


def run_solves(solver, steps, warmup, rtol=1e-6):
    import torch

    x = None
    for _ in range(warmup):
        x, st = solver.solve(rtol=rtol, out=x)
    torch.cuda.synchronize()
    times, iters, stats = [], [], None
    for _ in range(steps):
        t0 = time.perf_counter()
        x, stats = solver.solve(rtol=rtol, out=x)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        iters.append(sum(s.iterations for s in stats))
    return x, stats, times, iters


def kernel_roofline(solver, nrhs, prec_idx, n_nodes, x, solves):
    """Per-kernel average launch duration inside real solves of the workload:
    `solves` solves with the library's event tracing on (HIP events on the
    solver's stream around every fine-level launch, steps launched directly
    instead of replayed as a graph), then algorithmic bytes / duration.  The
    durations are the event-bracketed averages as measured; the bracket's own
    cost (events around a launch whose workgroups all exit at once) is
    returned beside them, not subtracted."""
    solver.set_option("trace", 1)
    for _ in range(solves):
        solver.solve(rtol=1e-6, out=x)
    ms, cnt = solver.kernel_times()
    solver.set_option("trace", 0)
    bracket = ms[6]
    rows = {}
    for kid, (name, per_iter, _, _) in KERNELS.items():
        algo = kernel_bytes(kid, prec_idx, nrhs) * n_nodes
        rows[name] = {"ms": ms[kid], "launches": cnt[kid], "per_iter": per_iter,
                      "bytes": int(algo), "GBs": algo / (ms[kid] * 1e-3) / 1e9 if ms[kid] > 0 else None}
    dom = max(rows, key=lambda k: rows[k]["ms"] * rows[k]["per_iter"])
    return dom, rows, bracket


# the oracle's peak host memory per node during one Bi-CGSTAB step (complex128
# Krylov vectors, the multigrid levels and NumPy's temporaries: 292 B measured
# on a 257^3 cube), with a margin
ORACLE_BYTES_PER_NODE = 400
# largest cube the oracle sample runs on (one complex128 step of the oracle
# grows linearly with the nodes: 0.7 s at 129^3, 5.7 s at 257^3 on a 16-core
# host of the GPU machine, so about 46 s at 513^3)
ORACLE_MAX_CUBE = 513


def cpu_baseline(wl, nodes, n_iter):
    """The CPU oracle on a bounded sample of the workload: n_iter complex128
    Bi-CGSTAB steps (set-up excluded), BLAS held to one thread.  For a cube
    larger than ORACLE_MAX_CUBE, or than the host's free memory holds, the
    sample is the largest 2^j + 1 cube below it with the same kh, boundary
    condition and centre source (one level fewer per halving); the oracle's
    time per DoF-iteration does not depend on the grid size."""
    import oracle as O
    import workloads as W
    from oracle.discretization import Level
    from oracle.multigrid import build_hierarchy, vcycle

    from threadpoolctl import threadpool_limits

    note = ""
    if wl.shape[0] == wl.shape[1] == wl.shape[2] and wl.shape[0] > 65 and np.all(wl.k == wl.k.flat[0]):
        import psutil

        avail = psutil.virtual_memory().available
        n, levels = wl.shape[0], wl.n_levels
        kh = float(wl.k.flat[0]) * wl.h
        while n > 65 and (n > ORACLE_MAX_CUBE or n ** 3 * ORACLE_BYTES_PER_NODE > avail):
            n, levels = (n - 1) // 2 + 1, levels - 1
        if n != wl.shape[0]:
            note = (f"; sample on the {n}^3 cube with the same kh = {kh:g}, boundary condition and centre "
                    f"source ({levels} levels) in place of {wl.shape[0]}^3, where one oracle step takes "
                    f"about {(wl.shape[0] - 1) ** 3 // (n - 1) ** 3} times as long "
                    f"(host memory free: {avail / 2**30:.0f} GiB)")
            wl = W.constant_cube(n, kh * (n - 1), wl.bc, n_levels=levels)
            nodes = wl.sources
    lvl = Level(wl.shape, wl.h, wl.k, wl.bc)
    hier = build_hierarchy(wl.k, wl.h, wl.bc, n_levels=wl.n_levels)
    b = O.point_source_rhs(wl.shape, wl.h, nodes[:1])[0]
    # NumPy's element-wise work is single-threaded; the BLAS / LAPACK calls are
    # held to one thread as well, so the whole sample runs on one core
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        O.bicgstab(lambda x: O.apply_A(x, lvl), lambda r: vcycle(r, hier), b, fixed_iterations=n_iter)
        dt = time.perf_counter() - t0
    return {"value": dof(wl) * n_iter / dt, "unit": "DoF-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_iter} complex128 Bi-CGSTAB step(s) of {wl.name}, one source, NumPy/SciPy "
                      f"single thread on a host of {os.cpu_count()} cores ({dt:.1f} s){note}"}


def beta2_sweep(args, wl, nodes, desc):
    """V- and F-cycle solves over the complex shift beta2 (mixed precision)."""
    import torch

    from paper_2308_06085_amd import Solver

    k = torch.from_numpy(wl.k).cuda()
    rows = []
    for beta2 in (-0.5, -0.6, -0.7, -0.8, -0.9, -1.0):
        for method in ("bicgstab", "idrs", "gmres"):
            for cyc in ("V", "F"):
                s = Solver(wl.shape, wl.h, bc=wl.bc, prec="mixed", cycle=cyc, beta=(1.0, beta2), method=method)
                s.set_model(k)
                s.set_point_sources(nodes)
                # at most 1200 products with A for Bi-CGSTAB and IDR(4); GMRES (restarted
                # every 200 steps, each step a pass over the basis) at most 400
                maxit = {"bicgstab": 600, "idrs": 1200, "gmres": 400}[method]
                # GMRES launches directly (nothing to warm up) and runs for seconds: one solve
                warm, reps = (0, 1) if method == "gmres" else (args.warmup, args.steps)
                x = None
                for _ in range(warm):
                    x, _ = s.solve(rtol=1e-6, maxit=maxit, out=x)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    x, st = s.solve(rtol=1e-6, maxit=maxit, out=x)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / reps
                rows.append({"beta2": beta2, "method": method, "cycle": cyc, "iterations": st[0].iterations,
                             "matvecs": st[0].matvecs, "status": st[0].status,
                             "relres_true": st[0].relres_true, "ms_per_solve": ms})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
                s.close()
                del x
    ok = [r for r in rows if r["status"] == "HH_OK"]
    best = min(ok, key=lambda r: r["ms_per_solve"])
    line = {
        "metric": "time to 1e-6 rel residual over beta2: Bi-CGSTAB, IDR(4) and GMRES, V- and F-cycle (mixed)",
        "value": best["ms_per_solve"], "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": best["ms_per_solve"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 cycle / c128 Krylov", "data": "synthetic",
        "config": {"workload": desc, "unknowns": dof(wl), "nrhs": 1, "rtol": 1e-6,
                   "max_products_with_A": 1200, "max_gmres_steps": 400, "precision": "mixed"},
        "best": best, "sweep": rows,
    }
    print(json.dumps(line), flush=True)


def variant_solves(args, wl, nodes, make, vres, combos):
    """The timed solves again with the other Krylov method / multigrid cycle."""
    import torch

    out = {}
    for method, cyc in combos:
        key = f"{method}+{cyc}"
        out[key] = {}
        for prec, v in vres.items():
            s = make(prec, method=method, cycle=cyc)
            x, stats, times, iters = run_solves(s, args.steps, args.warmup)
            t = float(np.sum(times))
            out[key][prec] = {
                "iterations": float(np.mean(iters)), "matvecs": int(np.mean([st.matvecs for st in stats])),
                "ms_per_step": 1e3 * t / args.steps,
                "relres_true_max": max(st.relres_true for st in stats),
                "status": sorted({st.status for st in stats}),
                "time_to_solution_speedup_vs_headline": v["ms_per_step"] / (1e3 * t / args.steps)}
            s.close()
            del x
            torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube513",
                    choices=["cube513", "wedge", "batched", "beta2_sweep", "closedoff129"])
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the F-cycle and IDR(4) solves of the wedge")
    ap.add_argument("--cycle", default="V", choices=["V", "F"],
                    help="preconditioner cycle of the headline solves (default V)")
    ap.add_argument("--method", default="bicgstab", choices=["bicgstab", "idrs", "gmres"],
                    help="Krylov method of the headline solves (default bicgstab; idrs = IDR(4); gmres = full GMRES)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the complex128 comparison solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="oracle Bi-CGSTAB steps of the cpu_baseline sample (default 1 on the cube, 8 otherwise)")
    ap.add_argument("--trace-solves", type=int, default=None,
                    help="event-traced solves behind the roofline (default 2 on the cube, else --steps)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch shapes with hh_autotune first (default for --workload batched)")
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON cache file of hh_autotune (read first, updated after measuring)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 1 GiB device buffer 3 times (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver keeps the whole grid on one device "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2308_06085_amd import Solver

    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        bbuf = torch.empty_like(a)
        for _ in range(3):
            bbuf.copy_(a)
        torch.cuda.synchronize()
        del a, bbuf
    if args.workload == "closedoff129":
        closed_off_runs(args)
        return
    wl, nodes, desc = make_workload(args.workload)
    if args.workload == "beta2_sweep":
        beta2_sweep(args, wl, nodes, desc)
        return
    nrhs = len(nodes)
    n_nodes = int(np.prod(wl.shape))
    k = torch.from_numpy(wl.k).cuda()

    tuned = {}

    def make(prec, method=None, cycle=None):
        s = Solver(wl.shape, wl.h, bc=wl.bc, prec=prec, n_levels=wl.n_levels, nrhs_max=nrhs,
                   cycle=cycle or args.cycle, method=method or args.method)
        s.set_model(k)
        s.set_point_sources(nodes)
        if args.autotune or args.workload == "batched":
            shapes = s.autotune(args.autotune_cache)
            tuned.setdefault(prec, shapes)  # the timed solves' shapes
        return s

    # progress lines on stderr (stdout carries only the result line)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    results = {}
    solutions = {}
    cube = args.workload == "cube513"
    traced = args.trace_solves if args.trace_solves is not None else (2 if cube else max(1, args.steps))
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        s = make(prec)
        # the cube's FP64 comparison: at most 5 timed solves after at most one
        # warm-up (its step count is deterministic), to keep the GPU time short
        reps, warm = ((min(args.steps, 5), min(args.warmup, 1)) if cube and prec == "fp64"
                      else (args.steps, args.warmup))
        x, stats, times, iters = run_solves(s, reps, warm)
        t = float(np.sum(times))
        it = float(np.mean(iters))
        # the library's own true residual ||b - A x|| / ||b|| after the solve (the
        # GPU tests hold it to the oracle's operator within 1e-9)
        rel = [s_.relres_true for s_ in stats]
        if args.method == "bicgstab":
            dom, rows, bracket = kernel_roofline(s, nrhs, 0 if prec == "fp64" else 1, n_nodes, x, traced)
        else:  # the library's in-solve kernel tracing covers the Bi-CGSTAB step only
            dom, rows, bracket = None, {}, None
        # bytes of the solves: every right-hand side's own bytes per step it
        # iterated, the shared k^2 / k bytes once per step of the longest one
        pi = 0 if prec == "fp64" else 1
        per_rhs, shared = step_bytes(pi, 1) - step_bytes(pi, 0), step_bytes(pi, 0)
        solve_bytes = n_nodes * (per_rhs * float(np.sum(iters)) + shared * reps * max(s_.iterations for s_ in stats))
        bpd = solve_bytes / (dof(wl) * float(np.sum(iters)))
        step_gbs = solve_bytes / t / 1e9
        results[prec] = {
            "hbm_per_iteration": {"bytes_per_dof": round(bpd, 1), "GBs": step_gbs,
                                  "frac": step_gbs / HBM_PEAK_GBS} if args.method == "bicgstab" else None,
            "value": dof(wl) * float(np.sum(iters)) / t,
            "ms_per_step": 1e3 * t / reps,
            "steps": reps, "warmup": warm,
            "iterations": it,
            "matvecs": int(sum(st.matvecs for st in stats)),
            "relres_true_max": max(rel),
            "status": sorted({st.status for st in stats}),
            "block": s.get_option("block"), "zb": s.get_option("zb"),
            "dominant": dom, "kernels": rows, "event_bracket_ms": bracket,
        }
        log(prec, json.dumps(results[prec]) if args.verbose else
            f"{results[prec]['ms_per_step']:.1f} ms per solve, {it} steps")
        s.close()
        solutions[prec] = x
        del x
        torch.cuda.empty_cache()
    # error of each solution against a tight FP64 solve (relative 2-norm, worst
    # right-hand side), outside the timed region
    ref_err = None
    if not args.no_fp64:
        s = make("fp64")
        xr, _ = s.solve(rtol=1e-10, maxit=20000)
        ref_err = {"ref_rtol": 1e-10}
        for prec, xs in solutions.items():
            e = [float(torch.linalg.vector_norm(xs[i] - xr[i]) / torch.linalg.vector_norm(xr[i]))
                 for i in range(nrhs)]
            ref_err[prec] = max(e)
        s.close()
        del xr
    solutions.clear()
    torch.cuda.empty_cache()
    fres = None
    if not args.no_variants and args.cycle == "V" and args.method == "bicgstab":
        if args.workload == "wedge":
            fres = variant_solves(args, wl, nodes, make, results,
                                  (("bicgstab", "F"), ("idrs", "V"), ("idrs", "F"), ("gmres", "V"), ("gmres", "F")))
        elif args.workload == "batched":
            fres = variant_solves(args, wl, nodes, make, results, (("bicgstab", "F"),))

    head = results["mixed"]
    dom = head["dominant"]
    row = head["kernels"].get(dom)
    traffic = None
    key = (dom, args.workload, "mixed")
    if key in TRAFFIC and TRAFFIC[key][1] == kernel_source_sha():
        traffic = TRAFFIC[key][0]
    roofline = None
    ref = streaming_reference(torch)
    if row is not None and row["GBs"]:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": row["GBs"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": row["GBs"] / HBM_PEAK_GBS, "traffic": traffic,
                    "algorithmic_bytes_per_launch": row["bytes"], "avg_ms": row["ms"],
                    "event_bracket_ms": head["event_bracket_ms"], "launches": row["launches"],
                    "traced_solves": traced, "frac_of_streaming_reference": row["GBs"] / ref["GBs"]}
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "DoF-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"c64 {args.cycle}-cycle / c128 Krylov",
        "data": "synthetic",
        "config": {"workload": desc, "unknowns": dof(wl), "nrhs": nrhs, "rtol": 1e-6,
                   "precision": "mixed", "cycle": args.cycle,
                   "method": {"idrs": "IDR(4)", "gmres": "GMRES"}.get(args.method, "Bi-CGSTAB"),
                   # the library's default for the mixed form: Bi-CGSTAB restarts from x
                   # each time the residual falls below another power of ten
                   "mixed_bicgstab_restarts": "at every power of ten of the residual"
                   if args.method == "bicgstab" else "none"},
        "iterations": head["iterations"],
        "relres_true_max": head["relres_true_max"],
        "hbm_per_iteration": head["hbm_per_iteration"],
        "roofline": roofline,
        "streaming_reference": ref,
        "kernels_mixed": {k_: {"ms": v["ms"], "GBs": v["GBs"] and round(v["GBs"], 1)}
                          for k_, v in head["kernels"].items()},
    }
    if "fp64" in results:
        f = results["fp64"]
        line["fp64"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "iterations": f["iterations"],
                        "steps": f["steps"], "warmup": f["warmup"],
                        "hbm_per_iteration": f["hbm_per_iteration"],
                        "relres_true_max": f["relres_true_max"], "dominant": f["dominant"],
                        "kernels": {k_: {"ms": v["ms"], "GBs": v["GBs"] and round(v["GBs"], 1)}
                                    for k_, v in f["kernels"].items()}}
        line["mixed_speedup_time_to_solution"] = f["ms_per_step"] / head["ms_per_step"]
        line["mixed_speedup_per_iteration"] = ((f["ms_per_step"] / f["iterations"])
                                               / (head["ms_per_step"] / head["iterations"]))
    if ref_err is not None:
        line["error_vs_fp64_reference"] = ref_err
    if tuned:
        line["autotuned_shapes"] = tuned
    if fres is not None:
        line["variants"] = fres
    if not args.no_cpu:
        log("cpu_baseline: timing the oracle")
        del k
        torch.cuda.empty_cache()
        n_iter = args.cpu_iters if args.cpu_iters is not None else (1 if cube else 8)
        line["cpu_baseline"] = cpu_baseline(wl, nodes, n_iter)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
