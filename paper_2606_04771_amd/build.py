"""Build the HIP library ``libtdvp.so`` (gfx950) in-tree with hipcc.

Usage: python -m paper_2606_04771_amd.build   (or build() from Python).
Every call recompiles the sources that changed (object timestamps) and
relinks; ``force=True`` recompiles everything.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtdvp.so")
SOURCES = ["symm.cpp", "plan.cpp", "abelian.cpp", "common.cpp", "capi_host.cpp", "tridiag.cpp", "capi_dev.cpp",
           "capi_u1.cpp",
           "krylov.cpp", "sweep.cpp", "gemm.hip", "vec.hip", "eig.hip", "noalloc.hip"]
# host sources that launch kernels or use HIP device types are compiled as HIP
HIP_CPP = ("capi_dev.cpp", "capi_u1.cpp", "krylov.cpp", "sweep.cpp")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def build(force=False, verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    hipcc = _hipcc()
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    headers.append(os.path.join(HERE, "..", "include", "tdvp.h"))
    hdr_time = max(os.path.getmtime(h) for h in headers)
    objs, cmds = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(OBJ, src + ".o")
        objs.append(obj)
        if (not force and os.path.exists(obj) and os.path.getmtime(obj) >= os.path.getmtime(path)
                and os.path.getmtime(obj) >= hdr_time):
            continue
        lang = ["-x", "hip"] if src.endswith(".hip") or src in HIP_CPP else []
        cmds.append([hipcc] + FLAGS + lang + ["-c", path, "-o", obj])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    jobs = max(1, min(len(cmds), len(os.sched_getaffinity(0)), 16))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", LIB + ".tmp"] + objs + [
        "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True)
