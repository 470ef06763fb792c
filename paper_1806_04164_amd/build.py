"""Build libpie.so (the C-ABI library) in-tree for gfx950 with hipcc.

Device translation units are compiled with -O3 for gfx950 with packed-FP32
instruction generation disabled; host-only units (mesh, tree, tables) with
-ffp-contract=off so that geometric predicates and box assignment are
reproducible bit for bit.  Run: python -m paper_1806_04164_amd.build
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpie.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

DEVICE_SOURCES = ["near.hip", "far.hip", "aux.hip", "op.hip"]
HOST_SOURCES = ["mesh_tree.cpp", "tables.cpp"]
ARCH = "gfx950"


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _common():
    return ["-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{os.path.dirname(HERE)}/include"]


def _compile(args):
    cmd, src = args
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r.stderr


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = []
    objs = []
    for src in DEVICE_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmd = [hipcc, "-x", "hip", "-O3", f"--offload-arch={ARCH}", "-mcode-object-version=5",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-munsafe-fp-atomics", *_common(), "-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append((cmd, src))
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmd = [hipcc, "-x", "c++", "-O2", "-ffp-contract=off", *_common(), "-c",
               os.path.join(CSRC, src), "-o", obj]
        jobs.append((cmd, src))
        objs.append(obj)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for msg in ex.map(_compile, jobs):
            if verbose and msg.strip():
                print(msg, file=sys.stderr)
    tmp = OUT + ".tmp"
    link = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
            "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
