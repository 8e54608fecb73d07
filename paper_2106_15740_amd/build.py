"""Builds the HIP library ``_lib/libqtn.so`` for gfx950 with hipcc (in-tree).

The kernels are split over several translation units (per element type and
executor set) that compile in parallel, then link into one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
OBJ_DIR = os.path.join(OUT_DIR, "obj")
LIB = os.path.join(OUT_DIR, "libqtn.so")

# (source, object name, extra defines)
UNITS = [
    ("plan.cpp", "plan", []),
    ("api.cpp", "api", []),
    ("kernels.hip", "kernels", []),
    ("kern_ops.hip", "ops_f32", ["-DQTN_REAL=float"]),
    ("kern_ops.hip", "ops_f64", ["-DQTN_REAL=double"]),
    ("kern_persist.hip", "pers_f32_n", ["-DQTN_REAL=float", "-DQTN_WIDE=false"]),
    ("kern_persist.hip", "pers_f32_w", ["-DQTN_REAL=float", "-DQTN_WIDE=true"]),
    ("kern_persist.hip", "pers_f64_n", ["-DQTN_REAL=double", "-DQTN_WIDE=false"]),
    ("kern_persist.hip", "pers_f64_w", ["-DQTN_REAL=double", "-DQTN_WIDE=true"]),
]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware float atomics on device memory
    "-munsafe-fp-atomics",
    "-Wall",
    "-Wno-unused-result",
]


def _hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _compile(unit, extra_flags):
    src, name, defs = unit
    obj = os.path.join(OBJ_DIR, name + ".o")
    cmd = [_hipcc(), *HIPCC_FLAGS, *extra_flags, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src} ({name}):\n" + res.stdout + res.stderr)
    return obj, res.stderr


def build(verbose: bool = False, out: str = LIB, extra_flags=(), jobs: int = 0) -> str:
    """Compile every translation unit (in parallel) and link the shared
    library; returns its path.  extra_flags go to every hipcc line (e.g.
    host-only sanitizers as ``-Xarch_host -fsanitize=...``)."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(u, list(extra_flags)), UNITS))
    if verbose:
        for _, err in results:
            if err.strip():
                print(err)
    tmp = out + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *extra_flags, *[o for o, _ in results], "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
