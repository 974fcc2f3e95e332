"""Build libmoma.so (HIP for gfx950) in place, next to this file.

Run as a script (python paper_2501_07535_amd/build.py) or through
__graft_entry__.build(); importing the package itself needs a built library.

Each source is compiled by hipcc in its own process (they run in parallel),
then linked into one shared library exporting the C ABI of include/moma.h.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmoma.so")
ARCH = os.environ.get("MOMA_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # unroll every `#pragma unroll` loop fully, however large the body: from 11
    # limbs on the default threshold leaves the loops over a radix-4 unit's
    # butterflies partly rolled, and indexing the unit's element array inside a
    # rolled loop puts the array in scratch memory
    "-mllvm", "-pragma-unroll-threshold=100000000",
    "-Wall", "-Wno-unused-function",
]

SOURCES = ["ntt_inst_g.hip", "ntt_inst_c.hip", "ntt_inst_h.hip", "ntt_inst_b.hip", "ntt_inst_e.hip", "ntt_inst_i.hip",
           "ntt_inst_a.hip", "ntt_inst_f.hip", "ntt_inst_d.hip", "blas.hip", "ntt.hip", "mlp.hip", "probe.hip",
           "noalloc.hip", "capi.cpp", "batch.cpp", "tune.cpp", "costmodel.cpp"]


def _compile(src: str) -> tuple[str, float]:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    return obj, time.time() - t0


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        done = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in done]
    if verbose:
        print("compile seconds:", ", ".join(f"{s} {t:.0f}" for s, (_, t) in zip(SOURCES, done)))
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
