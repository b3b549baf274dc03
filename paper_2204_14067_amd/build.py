"""Builds libbmg.so (the HIP kernels and the C ABI of include/bmg.h) for gfx950.

    python -m paper_2204_14067_amd.build

The library is placed next to this file, so it travels with the source tree.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libbmg.so")
# the row kernels of the sparse passes (rowpass.h) are instantiated once per
# element type pair in their own source, so the heavy sources compile in parallel
SOURCES = ["pass_f64.hip", "pass_f32.hip", "pass_bf16.hip", "kernels.hip", "api.hip", "linalg.cpp",
           "server.cpp"]
# every source that defines device code (hashed by bench.py to match counter records)
KERNEL_SOURCES = ["bmg_internal.h", "rowpass.h", "pass_f64.hip", "pass_f32.hip", "pass_bf16.hip",
                  "kernels.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions in the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def _compile(src: str, objdir: str, verbose: bool) -> str:
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
    return obj


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS") or os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir, verbose), SOURCES))
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("link of libbmg.so failed")
    os.replace(tmp, SO)
    return SO


def kernel_sources_sha256() -> str:
    """sha256 over the device-code sources, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


if __name__ == "__main__":
    print(build(verbose=True))
