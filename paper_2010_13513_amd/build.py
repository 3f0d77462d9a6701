"""Build libhhg.so in-tree with hipcc for gfx950.

Packed FP32 instructions are disabled for all device code
(-target-feature -packed-fp32-ops).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = ["api.hip", "kernels.hip", "mlp.hip", "fe_host.cpp"]
GEN_SRC = ["gen_stencils.cpp", "fe_host.cpp"]
GEN_OUT = os.path.join(HERE, "csrc", "generated", "stencils.inc")
LIB = os.path.join(HERE, "libhhg.so")
ARCH = os.environ.get("HHG_OFFLOAD_ARCH", "gfx950")


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


def build(verbose=True):
    generate(verbose)
    srcs = [os.path.join(HERE, "csrc", s) for s in SRC]
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-o", LIB + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
