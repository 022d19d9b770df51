"""Builds libcutbddc.so (HIP kernels for gfx950 + host C++) in-tree.

Every call recompiles all sources.  Compiler flags:
  * -ffp-contract=off: the kept-point test and the exact edge/ball tests
    decide integer data and must not be contracted into FMAs;
  * -Xclang -target-feature -Xclang -packed-fp32-ops: no packed FP32 ops.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libcutbddc.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"-I{INCLUDE}", f"-I{CSRC}",
          "-I/opt/rocm/include"]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HIP_SOURCES = ["integrate.hip", "indexing.hip", "operator.hip", "dense.hip", "bddc.hip", "noalloc.hip", "nitsche.hip",
               "manufactured.hip", "coarse_nd.hip"]
HOST_SOURCES = ["topology.cpp", "cutbddc.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {' '.join(cmd[:3])} ...")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([HIPCC, "-c", *COMMON, *DEVICE, os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([HIPCC, "-c", "-x", "c++", *COMMON, "-D__HIP_PLATFORM_AMD__",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    procs = [subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
             for j in jobs]
    failed = []
    for j, p in zip(jobs, procs):
        out, err = p.communicate()
        if p.returncode != 0:
            failed.append((j, out + err))
        elif verbose and err.strip():
            sys.stderr.write(err)
    if failed:
        for j, msg in failed:
            sys.stderr.write(" ".join(j) + "\n" + msg + "\n")
        raise RuntimeError("HIP build failed")
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "--offload-arch=" + ARCH, *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
