"""Build the gfx950 shared library ``libhh.so`` of this package in place.

    python -m paper_2308_06085_amd.build

Compiles every HIP source under ``csrc/`` with hipcc for gfx950 into one
shared library next to this file.  Packed FP32 instructions are disabled in
the device code (``-target-feature -packed-fp32-ops``); the multigrid passes
(``hh_mg_fused.hip``) are compiled with ``-ffp-contract=off``.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhh.so")
SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
ARCH = os.environ.get("HH_OFFLOAD_ARCH", "gfx950")
# The multigrid passes are compiled without implicit multiply-add contraction:
# they write their fused multiply-adds out, so every inlined copy of a loop
# body rounds alike and the results do not depend on z-blocks or regions.
EXTRA_FLAGS = {"hh_mg_fused.hip": ["-ffp-contract=off"]}


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile the library; returns its path.  Raises on any compiler error."""
    cc = hipcc()
    objs = []
    tmp = LIB + ".tmp"
    flags = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
             "-Wno-unused-result", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    def compile_one(src):
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [cc, *flags, *EXTRA_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        # the host pass does not know the device-only feature name: drop that line
        noise = [ln for ln in (r.stderr or "").splitlines() if "packed-fp32-ops" not in ln]
        return src, obj, r.returncode, noise

    # one hipcc per source, several at a time
    workers = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        results = list(pool.map(compile_one, SOURCES))
    for src, obj, rc, noise in results:
        if rc != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(noise))
        if verbose and noise:
            print("\n".join(noise), file=sys.stderr)
        objs.append(obj)
    # -z defs: a symbol no source defines fails the link instead of the first load
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Wl,-z,defs", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
