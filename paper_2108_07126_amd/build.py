"""Build the HIP library libparament.so in-tree for gfx950.

``python paper_2108_07126_amd/build.py`` (or ``build()``) compiles every
source under csrc/ with hipcc into paper_2108_07126_amd/libparament.so.
Run it as a script or load it by path: importing the package loads the
library, which may not exist yet.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libparament.so")
SOURCES = ["parament.cpp", "engine_mfma.hip", "engine_mfma_pair.hip", "engine_mfma_m6.hip", "engine_valu.hip", "engine_valu_f64_2.hip", "engine_valu_f64_4.hip",
           "engine_valu_f32_2.hip", "engine_valu_f32_4.hip", "engine_grad.hip", "engine_batch.hip", "engine_grape.hip", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _compile(src: str, obj: str, verbose: bool) -> None:
    cmd = [HIPCC, *FLAGS, "-c", "-I", os.path.join(HERE, "..", "include"), src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed compiling {os.path.basename(src)}")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel) and link libparament.so."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    jobs = jobs or min(len(srcs), os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_compile, s, o, verbose) for s, o in zip(srcs, objs)]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libparament.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
