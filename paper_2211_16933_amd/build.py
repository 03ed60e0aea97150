"""Build libelb.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: python -m paper_2211_16933_amd.build   (or call build()).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libelb.so")
SOURCES = ["elb.hip", "host_math.cpp"]
HEADERS = ["elb_kernels.h", "host_math.h"]

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # packed FP32 instructions are kept out of every kernel on this target
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libelb.so")
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    files = SOURCES + HEADERS
    paths = [os.path.join(CSRC, f) for f in files] + [os.path.join(os.path.dirname(HERE), "include", "elb.h")]
    return any(os.path.getmtime(p) > t for p in paths)


if __name__ == "__main__":
    print(build(verbose=True))
