"""Builds libsans.so (HIP, gfx950) in-tree with hipcc.

The per-model kernel instances are spread over several translation units
(sans_kinds.hip once per kind group, the batched kernel, the surrogate
kernels), compiled in parallel to objects under _build/ and linked into one
shared library.

Usage: python -m paper_2501_06054_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
SO = os.path.join(HERE, "libsans.so")
KIND_GROUPS = 8

# (source, extra defines, object name)
UNITS = ([("sans_lib.hip", [], "sans_lib.o"),
          ("sans_batch.hip", [], "sans_batch.o"),
          ("sans_sur.hip", [], "sans_sur.o"),
          ("sans_mlp.hip", [], "sans_mlp.o"),
          ("sans_host_math.cpp", [], "sans_host_math.o")]
         + [("sans_kinds.hip", [f"-DSANS_KIND_GROUP={g}"], f"sans_kinds_{g}.o") for g in range(KIND_GROUPS)])

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # hardware FP64 atomics (global_atomic_add_f64 / ds_add_f64) instead of CAS loops
    "-munsafe-fp-atomics",
    # no packed FP32 (v_pk_*_f32) code generation
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep constant materialisation inside the neutron loops: hoisting it out
    # (machine LICM) keeps dozens of FP64 constants live in VGPRs and halves
    # the waves per SIMD of the grid-stride trace kernels
    "-mllvm", "-disable-machine-licm",
    "-Wno-unused-command-line-argument",
]

LINK = ["--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-rpath,/opt/rocm/lib"]


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16, len(UNITS)))


def _compile(unit, verbose: bool):
    src, defs, obj = unit
    cmd = [HIPCC, *FLAGS, *defs, "-c", "-o", os.path.join(OBJ, obj), os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return unit, r


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    failed = [(u, r) for u, r in results if r.returncode != 0]
    for u, r in failed:
        sys.stderr.write(f"--- {u[0]} {' '.join(u[1])}\n" + r.stdout + r.stderr)
    if failed:
        raise RuntimeError("hipcc failed building libsans.so")
    tmp = SO + ".tmp"
    cmd = [HIPCC, *LINK, "-o", tmp, *[os.path.join(OBJ, u[2]) for u in UNITS]]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libsans.so")
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
