"""Build librh.so (HIP for gfx950) in the package directory.

Usage: python paper_0908_2654_amd/build.py  (runs without importing the package,
which would load the library being rebuilt).
Each source is compiled to an object under _build/ and linked with hipcc.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = ["csrc/rh_kernels.hip", "csrc/rh_advect.hip", "csrc/rh_blocks.hip", "csrc/rh_noalloc.hip",
           "csrc/rh_groups.hip",
           "csrc/rh_host.cpp", "csrc/rh_groups_host.cpp"]
LIB = os.path.join(PKG, "librh.so")
ARCH = os.environ.get("RH_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc"),
         # no packed FP32 instructions in any device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# ROCTx: the library marks its step phases as profiler ranges
LINK = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        out = _run([hipcc, *FLAGS, "-c", os.path.join(PKG, src), "-o", obj])
        if verbose and out.strip():
            print(out)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, *LINK, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
