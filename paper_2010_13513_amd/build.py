"""Build libhhg.so in-tree with hipcc for gfx950.

Each source is compiled to an object file in parallel, then linked.  Packed
FP32 instructions are disabled for all device code
(-target-feature -packed-fp32-ops).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = ["api.hip", "kernels.hip", "mlp.hip", "umesh.hip", "ukernels.hip", "fe_host.cpp"]
GEN_SRC = ["gen_stencils.cpp", "fe_host.cpp"]
GEN_OUT = os.path.join(HERE, "csrc", "generated", "stencils.inc")
OBJ_DIR = os.path.join(HERE, "csrc", "generated", "obj")
LIB = os.path.join(HERE, "libhhg.so")
ARCH = os.environ.get("HHG_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def generate(verbose=True):
    """Compile and run the host stencil generator (plain C++, g++)."""
    gen = os.path.join(HERE, "csrc", "generated", "gen_stencils")
    os.makedirs(os.path.dirname(gen), exist_ok=True)
    cmd = [os.environ.get("CXX", "g++"), "-O2", "-std=c++17", "-o", gen] + \
        [os.path.join(HERE, "csrc", s) for s in GEN_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    subprocess.run([gen, GEN_OUT + ".tmp"], check=True)
    os.replace(GEN_OUT + ".tmp", GEN_OUT)


def _compile(src, verbose):
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc(), f"--offload-arch={ARCH}"] + FLAGS + ["-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose=True):
    generate(verbose)
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = [os.path.join(HERE, "csrc", s) for s in SRC]
    jobs = min(len(srcs), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
