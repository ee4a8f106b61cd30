"""Compile the HIP sources of the library into ``libtk.so`` (gfx950), in-tree.

Each source is compiled to an object in parallel, then linked.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libtk.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("TK_OFFLOAD_ARCH", "gfx950")
SOURCES = ["tk_pass_dd.hip", "tk_pass_f64.hip", "tk_pass_f32.hip", "tk_contract.hip", "tk_batch.hip", "tk_build.hip",
           "tk_dense.hip", "tk_predict.hip", "tk_vec.hip", "tk_hess.hip", "tk_abi.hip", "tk_host.cpp"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-munsafe-fp-atomics", "-ffp-contract=off"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off"]
# Per-source additions: the batched MFMA pass adds its matrix-core results with
# vector instructions, and the build's sixteen accumulators per wave would
# otherwise sit in AGPRs beside as many VGPRs (one wave per SIMD): both keep
# their MFMA accumulators in VGPRs.
EXTRA_FLAGS = {"tk_batch.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
               "tk_build.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _up_to_date(src: str, obj: str) -> bool:
    """The object is newer than its source and than every header of csrc/ and
    include/ (a coarse rule: any header change rebuilds everything)."""
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)]
    deps += [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    inc = os.path.join(os.path.dirname(HERE), "include")
    deps += [os.path.join(inc, h) for h in os.listdir(inc) if h.endswith(".h")]
    return all(os.path.getmtime(p) < t for p in deps)


def _compile(src: str, changed_only: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    if changed_only and _up_to_date(src, obj):
        return obj
    if src.endswith(".cpp"):   # host-only C++ (planning, small dense algebra)
        cmd = [shutil.which("g++") or "g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    else:
        cmd = [hipcc(), *FLAGS, *EXTRA_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False, changed_only: bool = False) -> str:
    """Compile every source (changed_only: only those whose object is older
    than the source or a header) and link libtk.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, changed_only), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}", file=sys.stderr)
    return OUT


if __name__ == "__main__":
    build(verbose=True, changed_only="--changed" in sys.argv[1:])
