"""Sanitizer builds for the CPU test suite (AddressSanitizer + UndefinedBehaviorSanitizer).

* the oracle with its driver (gcc);
* the library's host code: every source compiled by hipcc with the
  sanitizers on the host side only (each -fsanitize= behind -Xarch_host; the
  gfx950 device code is built as usual), linked with the ABI driver by clang.

Everything goes to a directory the caller names; nothing is written in-tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1309_0551_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_oracle(out: str) -> str:
    exe = os.path.join(out, "oracle_driver")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "oracle", "lgt_oracle.c"), os.path.join(HERE, "oracle_driver.c"),
                    "-o", exe, "-lm"], check=True)
    return exe


def _sources():
    import importlib.util

    spec = importlib.util.spec_from_file_location("_lgt_build", os.path.join(ROOT, "paper_1309_0551_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.SOURCES


def build_abi(out: str, jobs: int = 8) -> str:
    objs = []

    def one(src):
        obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", INCLUDE,
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN_HOST, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = ["-x", "hip"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout}{r.stderr}")
        return obj

    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(one, _sources()))
    so = os.path.join(out, "liblgt_san.so")
    subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *SAN_HOST, "-o", so, *objs], check=True)
    exe = os.path.join(out, "abi_driver")
    subprocess.run([CLANG, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", INCLUDE, os.path.join(HERE, "abi_driver.c"), so, "-Wl,-rpath," + out, "-o", exe],
                   check=True)
    return exe
