"""Build libtumorgrad.so (HIP, gfx950) in the package directory.

Compiles the two precision translation units and the host C-ABI layer with
hipcc in parallel and links them into one shared library.  Always rebuilds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libtumorgrad.so")

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
DEV_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# The host layers are plain C++ against the HIP runtime API (no device code).
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HOST_FLAGS = ["-x", "c++", "-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__",
              f"-I{ROCM}/include", "-Wall", "-Werror=unused-result"]

GRIDS = (8, 16, 32, 64, 128, 256)
# one translation unit per (precision, grid size), plus the host layers
UNITS = ([("tg_inst.hip", DEV_FLAGS + [f"-DTG_INST_FP64={p}", f"-DTG_N={n}"], f"tg_inst_{p}_{n}")
          for p in (0, 1) for n in GRIDS]
         + [("tg_probe.hip", DEV_FLAGS, "tg_probe"), ("tg_static.hip", DEV_FLAGS, "tg_static"),
            ("tg_dispatch.cpp", HOST_FLAGS, "tg_dispatch"), ("tg_api.cpp", HOST_FLAGS, "tg_api")])


def _compile(src: str, flags: list[str], stem: str) -> str:
    obj = os.path.join(BUILD, stem + ".o")
    cmd = [HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    workers = max(1, min(len(UNITS), os.cpu_count() or 1, 16))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda u: _compile(*u), UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
