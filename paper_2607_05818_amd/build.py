"""Build libreff.so (HIP for gfx950) in-tree with hipcc.

Run as ``python -m paper_2607_05818_amd.build``; the repository's entry
module calls ``build()`` too.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libreff.so")

SOURCES = ["reff_api.cpp", "reff_kernels.hip", "grid_pairs.hip", "reduced_pairs.hip", "ir_drop.hip",
           "selinv.hip", "selinv_plan.cpp", "stream_probe.hip", "surrogate_api.cpp", "surrogate_kernels.hip",
           "coef_prep.hip"]

# Packed FP32 arithmetic is disabled for every HIP translation unit.
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def torch_lib_dir():
    """Directory of the HIP runtime that PyTorch loads.  libreff links that
    same runtime so that torch-allocated buffers and streams are valid in
    the library (two HIP runtimes in one process do not share devices)."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        return None
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *HIP_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return obj, subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, SOURCES))
    objs = []
    for src, (obj, r) in zip(SOURCES, results):
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        objs.append(obj)
    tmp = LIB + ".tmp"
    tl = torch_lib_dir()
    if tl:
        # Plain host link against torch's runtime (hipcc would add the
        # system libamdhip64 as well).
        cmd = ["g++", "-shared", "-fPIC", *objs, "-o", tmp, f"-L{tl}", "-l:libamdhip64.so",
               f"-Wl,-rpath,{tl}", "-Wl,--no-undefined"]
    else:
        cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libreff.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
