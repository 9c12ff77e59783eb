"""Build libibdvm.so for gfx950: HIP kernels with hipcc, host code with g++.

Run as ``python -m paper_2512_20252_amd.csrc.build`` or through
``__graft_entry__.build()``; objects go to ``_build/`` next to the package,
the library to ``paper_2512_20252_amd/libibdvm.so``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libibdvm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             # no packed FP32 instructions anywhere in the device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
              "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")]
INCLUDES = ["-I" + os.path.join(ROOT, "include"), "-I" + HERE]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    k_obj = os.path.join(BUILD, "kernels.o")
    # the FP64 2D update in its own unit, scheduled for instruction-level
    # parallelism (about 6 % faster there, slower for the other kernels)
    k64_obj = os.path.join(BUILD, "kernels_update2d_f64.o")
    jobs = [[HIPCC] + HIP_FLAGS + INCLUDES + ["-c", os.path.join(HERE, "kernels.hip"), "-o", k_obj],
            [HIPCC] + HIP_FLAGS + INCLUDES + ["-DIBDVM_FP64_UPDATE2D_UNIT", "-mllvm", "-amdgpu-sched-strategy=max-ilp",
                                              "-c", os.path.join(HERE, "kernels.hip"), "-o", k64_obj]]
    procs = []
    for cmd in jobs:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    codes = [p.wait() for p in procs]
    for cmd, code in zip(jobs, codes):
        if code:
            raise subprocess.CalledProcessError(code, cmd)
    objs = [k_obj, k64_obj]
    for src in ("geometry.cpp", "ibdvm.cpp", "server.cpp"):
        o = os.path.join(BUILD, src.replace(".cpp", ".o"))
        _run(["g++"] + HOST_FLAGS + INCLUDES + ["-c", os.path.join(HERE, src), "-o", o], verbose)
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
