"""Build step: compile the gfx950 HIP sources into paper_2305_18663_amd/libsbp.so."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsbp.so")
SOURCES = ["sbp_prims.hip", "sbp_sparse.hip", "sbp_dense.hip", "sbp_engine.hip", "sbp_dcsbp.hip"]
ARCH = os.environ.get("SBP_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-file additions.  The dense tier's kernels wait on dependent loads;
# scheduling for instruction-level parallelism measured 1% faster on the
# 200k-vertex sweep (evaluation 66.8 against 67.5-67.8 us), results unchanged.
FILE_FLAGS = {"sbp_dense.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}


def flags_of(src: str) -> list:
    return FLAGS + FILE_FLAGS.get(src, [])


def _compile(src: str, out_dir: str) -> str:
    obj = os.path.join(out_dir, src.replace(".hip", ".o"))
    cmd = ["hipcc", *flags_of(src), "-I", os.path.join(HERE, "..", "include"), "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as pool:
        objs = list(pool.map(lambda s: _compile(s, out_dir), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
