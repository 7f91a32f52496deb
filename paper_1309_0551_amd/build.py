"""Build liblgt.so (HIP, gfx950) in-tree.

Every source is compiled by hipcc for gfx950 only; the shared library is
written next to this file, where the Python binding loads it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
SO = os.path.join(HERE, "liblgt.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["dslash.hip", "blas.hip", "force.hip", "probe.hip", "mrhs.hip", "batch_cg.hip", "routines.hip", "hmc.hip", "fatten.hip", "noalloc.hip", "mcg.hip", "solver.cpp", "tune.cpp", "batch.cpp", "mcg_host.cpp", "hmc_abi.cpp", "abi.cpp"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# Packed FP32 instructions (v_pk_{add,mul,fma}_f32) are kept out of the code
# objects: some of their forms have given silently wrong results on these
# parts, and the compiler would otherwise form them from float / float2 code.
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", INCLUDE,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _compile(src: str) -> tuple[str, list[str]]:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    return obj, cmd


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    pending = [_compile(s) for s in SOURCES]
    while pending or procs:
        while pending and len(procs) < jobs:
            obj, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((obj, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        obj, cmd, p = procs.pop(0)
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the GPU target feature; that warning is harmless
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed ({p.returncode}): {' '.join(cmd)}\n{text}")
        if verbose and lines:
            print("\n".join(lines), flush=True)
    tmp = SO + ".tmp"
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
