"""Build libpeers.so in-tree: host C++ with g++, HIP kernels with hipcc for gfx950.

Usage: ``python -m paper_2606_31535_amd.build_lib`` (or ``build()`` from Python).
Always rebuilds every object. The library lands in ``paper_2606_31535_amd/_lib/``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_lib")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(OUT, "libpeers.so")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-march=x86-64-v3", "-Wall", "-Wno-unused-function",
              "-I" + os.path.join(ROOT, "include")]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-D__HIP_PLATFORM_AMD__",
             # no packed FP32 instructions anywhere in device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # keep MFMA accumulators in ordinary VGPRs (no AGPR copies in loops)
             "-mllvm", "-amdgpu-mfma-vgpr-form=1",
             "-I" + os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def sources():
    host = sorted(glob.glob(os.path.join(CSRC, "host", "*.cpp")))
    hip = sorted(glob.glob(os.path.join(CSRC, "hip", "*.hip")))
    return host, hip


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OUT, exist_ok=True)
    if os.path.isdir(OBJ):
        shutil.rmtree(OBJ)
    os.makedirs(OBJ, exist_ok=True)
    host, hip = sources()
    cmds = []
    objs = []
    for src in host:
        o = os.path.join(OBJ, "host_" + os.path.basename(src) + ".o")
        cmds.append(["g++"] + HOST_FLAGS + ["-c", src, "-o", o])
        objs.append(o)
    for src in hip:
        o = os.path.join(OBJ, "hip_" + os.path.basename(src) + ".o")
        cmds.append([HIPCC] + HIP_FLAGS + ["-c", src, "-o", o])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", "-fPIC", "-o", tmp] + objs + ["-pthread", f"-L{ROCM}/lib", "-lamdhip64"]
    _run(link)
    os.replace(tmp, LIB)
    shutil.rmtree(OBJ, ignore_errors=True)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
