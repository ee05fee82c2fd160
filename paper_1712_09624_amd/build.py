"""Builds the HIP library ``libckpp.so`` for gfx950 in-tree.

    python -m paper_1712_09624_amd.build
"""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libckpp.so")
SOURCES = ["ckpp_api.hip", "ckpp_lookup.hip", "ckpp_plan.hip", "ckpp_plan_timed.hip",
           "ckpp_serve.hip", "ckpp_update.hip", "ckpp_aux.hip"]
ARCH = os.environ.get("CKPP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False) -> str:
    """Compiles every HIP source (in parallel, one hipcc per source) and links
    them into one shared library (always rebuilds)."""
    import concurrent.futures
    import tempfile
    flags = [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # no packed fp32 instructions anywhere (the kernels are integer-only)
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-I", INCLUDE,
    ]
    with tempfile.TemporaryDirectory(prefix="ckpp_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]

        def compile_one(i):
            cmd = [hipcc()] + flags + ["-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
            return subprocess.run(cmd, capture_output=True, text=True)

        workers = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
        with concurrent.futures.ThreadPoolExecutor(workers) as pool:
            results = list(pool.map(compile_one, range(len(SOURCES))))
        for src, r in zip(SOURCES, results):
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + r.stdout + r.stderr)
            if verbose and r.stderr:
                print(r.stderr)
        tmp = LIB + ".tmp"
        r = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs,
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
