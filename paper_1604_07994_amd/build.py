"""Build the HIP library libiss.so in-tree for gfx950.

Usage: python -m paper_1604_07994_amd.build   (or build() from Python)
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libiss.so")
BUILD = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# packed FP32 instructions are disabled for all device code
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-ffp-contract=fast", "-munsafe-fp-atomics"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    jobs = []
    for src, dev in (("iss_kernels.hip", True), ("iss_net.hip", True), ("iss_krylov.hip", True),
                     ("iss_p1p0.hip", True), ("iss_host.cpp", False)):
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC] + COMMON + ["-x", "hip"] + DEVICE_FLAGS
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append(cmd)
        objs.append(obj)
    procs = []
    for cmd in jobs:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    for pr, cmd in zip(procs, jobs):
        if pr.wait() != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd))
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fopenmp", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
