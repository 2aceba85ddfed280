"""Builds libcsrk.so in-tree: host C++ with g++, HIP sources with hipcc for gfx950.

    python -m paper_2203_05096_amd.build          # build (always recompiles)
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "lib")
LIB = os.path.join(OUT_DIR, "libcsrk.so")
BUILD_DIR = os.path.join(ROOT, "_build", "csrk")

HOST_SOURCES = ["host/graph.cpp", "host/csr.cpp", "host/tune.cpp", "host/cpu_spmv.cpp"]
HIP_SOURCES = ["device/forward.hip", "device/adjoint.hip", "device/batch.hip", "device/util.hip", "device/cg.hip",
               "capi.hip"]

ARCH = os.environ.get("CSRK_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX_HOST", shutil.which("g++") or "g++")

# Packed FP32 instructions are kept out of generated code on purpose.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-fopenmp", "-Wall", "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def _obj(src):
    return os.path.join(BUILD_DIR, src.replace("/", "_") + ".o")


def _source_digest() -> str:
    """Digest of every source and header the library is built from."""
    import hashlib
    h = hashlib.sha256()
    for d in (CSRC, os.path.join(ROOT, "include")):
        for base, _, files in sorted(os.walk(d)):
            for f in sorted(files):
                if f.endswith((".hip", ".hpp", ".cpp", ".h")):
                    p = os.path.join(base, f)
                    h.update(p.encode())
                    h.update(open(p, "rb").read())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    os.makedirs(OUT_DIR, exist_ok=True)
    # hipcc compiles each file twice (device, then host) and reads the sources
    # each time: a source edited during the build would leave objects (and the
    # two halves of one object) from different versions.  Refuse that build.
    before = _source_digest()
    jobs = []
    for s in HOST_SOURCES:
        jobs.append([CXX, *HOST_FLAGS, "-c", os.path.join(CSRC, s), "-o", _obj(s)])
    for s in HIP_SOURCES:
        jobs.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", _obj(s)])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr, file=sys.stderr)
    if _source_digest() != before:
        raise RuntimeError("sources changed while the library was being built; build again")
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp,
          *[_obj(s) for s in HOST_SOURCES + HIP_SOURCES], "-lgomp"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
