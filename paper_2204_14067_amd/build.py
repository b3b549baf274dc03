"""Builds libbmg.so (the HIP kernels and the C ABI of include/bmg.h) for gfx950.

    python -m paper_2204_14067_amd.build

The library is placed next to this file, so it travels with the source tree.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libbmg.so")
SOURCES = ["kernels.hip", "api.hip", "linalg.cpp", "server.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions in the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc"] + FLAGS + ["-c", os.path.join(HERE, "csrc", src), "-o", obj]
        if src.endswith(".cpp"):   # host-only C++ (no device code)
            cmd = ["hipcc", "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + \
                [f for f in FLAGS if not f.startswith("--offload")
                 and f not in ("-Xclang", "-target-feature", "-packed-fp32-ops")] \
                + ["-c", os.path.join(HERE, "csrc", src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stderr)
            raise RuntimeError("compilation of %s failed" % src)
        objs.append(obj)
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("link of libbmg.so failed")
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
