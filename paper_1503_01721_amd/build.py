"""Build libdvmat.so (HIP for gfx950) in-tree.

    python -m paper_1503_01721_amd.build        # or __graft_entry__.build()

Every HIP translation unit is compiled with packed-FP32 instructions
disabled (-packed-fp32-ops); the host pass warns that it does not know the
feature, which is harmless.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libdvmat.so")
ARCH = os.environ.get("DVMAT_OFFLOAD_ARCH", "gfx950")

SOURCES = ["ddc_host.cpp", "spmv.hip", "spmv_panel.hip", "select.hip", "machine.hip", "bb.hip", "da.hip"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          f"-I{os.path.join(ROOT, 'include')}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          ]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libdvmat)")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l
                    and "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


def build(verbose: bool = True, jobs: int = 4) -> str:
    """Compile every source and link libdvmat.so; returns the library path."""
    cc = hipcc()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    t0 = time.time()
    procs, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        if src.endswith(".hip"):
            cmd = [cc, "-x", "hip", *DEVICE, *COMMON, "-c", path, "-o", obj]
        else:
            cmd = [cc, *COMMON, "-c", path, "-o", obj]
        procs.append(cmd)
    # compile in parallel
    running = []
    for cmd in procs:
        if verbose:
            print(" ".join(cmd), flush=True)
        running.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        if len(running) >= jobs:
            _wait(running.pop(0), verbose)
    for r in running:
        _wait(r, verbose)
    tmp = LIB + ".tmp"
    _run([cc, *DEVICE, "-shared", "-fPIC", "-pthread", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


def _wait(item, verbose):
    cmd, p = item
    out, _ = p.communicate()
    out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l
                    and "not a recognized feature" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
