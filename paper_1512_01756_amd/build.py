"""Build libsmpm_schur.so in place: host setup with g++, device code with
hipcc for gfx950.  `python -m paper_1512_01756_amd.build` rebuilds."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsmpm_schur.so")
BUILD = os.path.join(HERE, "_build")

HOST_SOURCES = ["dense.cpp", "setup_host.cpp", "persist.cpp"]
DEVICE_SOURCES = ["smpm.hip", "setup_dev.hip"]
ARCH = os.environ.get("SMPM_OFFLOAD_ARCH", "gfx950")


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (needs ROCm)")


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    host_flags = ["-O3", "-fPIC", "-std=c++17", "-mavx2", "-mfma", "-Wall", "-Wno-unused-function",
                  "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["g++", *host_flags, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    hipcc = _hipcc()
    dev_flags = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for src in DEVICE_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([hipcc, *dev_flags, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lrocsolver", "-lrocblas",
          "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
