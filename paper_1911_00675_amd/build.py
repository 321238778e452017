"""Build libpmh.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1911_00675_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpmh.so")
SOURCES = ["pmh_kernels.hip", "pmh_runtime.cpp", "pmh_autotune.cpp", "pmh_server.cpp"]

# Strict IEEE binary64 (no contraction, no fast math: signatures must match the
# CPU reference bit for bit); packed FP32 instructions disabled.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fno-fast-math", "-Wall", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, stats: bool = False) -> str:
    """Compile libpmh.so; stats=True builds the event-counting variant
    libpmh_stats.so (-DPMH_STATS) used for schedule analysis only."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = FLAGS + (["-DPMH_STATS"] if stats else [])
    lib = os.path.join(HERE, "libpmh_stats.so") if stats else LIB
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + (".stats.o" if stats else ".o"))
        cmd = [hipcc] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc] + flags + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
                          + ["-lpthread"])
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, stats="--stats" in sys.argv))
