"""Compile the HIP library (csrc/) for gfx950 into libwsmul.so, in-tree.

Every translation unit is compiled with hipcc for --offload-arch=gfx950 with
packed-FP32 instructions disabled, then linked into one shared library that
exports only the C-ABI declared in include/wsmul.h.  The feature flag reaches
the host pass too, which warns that it does not know it and ignores it (the
clang driver forwards no -Xclang argument to the device pass alone).
"""
import concurrent.futures
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libwsmul.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
          "-Wall", "-Wno-unused-result", "-fvisibility=hidden"]

SOURCES = ["plan.cpp", "capi.cpp", "autotune.cpp", "batch.cpp", "digit_temps.cpp", "kernels.hip",
           "limbs.hip"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    # Every unit is HIP: the C++ ones hold host code and the static device
    # scratch of the no-allocation entry point.
    cmd = [HIPCC, "-x", "hip"] + COMMON + ["-c", path, "-o", obj]
    subprocess.run(cmd, check=True)
    return obj


def build(jobs: int = 8) -> str:
    """Compile every source and link libwsmul.so; return its path."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build())
