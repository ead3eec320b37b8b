"""Builds libsans.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2501_06054_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libsans.so")
SOURCES = ["sans_lib.hip", "sans_mlp.hip", "sans_host_math.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # hardware FP64 atomics (global_atomic_add_f64 / ds_add_f64) instead of CAS loops
    "-munsafe-fp-atomics",
    # no packed FP32 (v_pk_*_f32) code generation
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep constant materialisation inside the neutron loops: hoisting it out
    # (machine LICM) keeps dozens of FP64 constants live in VGPRs and halves
    # the waves per SIMD of the grid-stride trace kernels
    "-mllvm", "-disable-machine-licm",
    "-Wno-unused-command-line-argument",
    "-Wl,-rpath,/opt/rocm/lib",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = SO + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libsans.so")
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
