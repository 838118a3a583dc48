"""Compile the gfx950 HIP library (libgearrt.so) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgearrt.so")
SOURCES = ["rt_api.hip", "rt_build.hip", "rt_step.hip", "rt_step32.hip", "rt_adjoint.hip",
           "rt_adjoint32.hip", "rt_bins.hip", "rt_hll.hip",
           "rt_absorb.hip", "rt_drift.hip",
           "rt_ivanova.hip"]
ARCH = os.environ.get("GEARRT_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
]


def _compile(src: str, bdir: str = BUILD, defines=()) -> str:
    obj = os.path.join(bdir, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, lib: str = LIB, defines=()) -> str:
    """Compile every source and link `lib`.  `defines` (NAME=VALUE strings) set
    the tuning macros of the kernels (tile shapes, groups per wave); a build
    with non-default macros goes to its own object folder and library path."""
    bdir = BUILD if not defines else os.path.join(BUILD, "_".join(sorted(defines)).replace("=", "-"))
    os.makedirs(bdir, exist_ok=True)
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda s: _compile(s, bdir, defines), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib} in {time.time() - t0:.1f} s", file=sys.stderr)
    return lib


if __name__ == "__main__":
    build(verbose=True)
