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
# (source, object name, extra flags); .cpp sources with HIP calls go through
# hipcc as host C++, the pure-host linear algebra through g++ (twice: baseline
# and x86-64-v3, chosen at run time by linalg_dispatch.cpp)
SOURCES = [("pass_f64.hip", "pass_f64", []), ("pass_f32.hip", "pass_f32", []),
           ("pass_bf16.hip", "pass_bf16", []), ("kernels.hip", "kernels", []),
           ("colpass.hip", "colpass", []), ("rke.hip", "rke", []), ("noalloc.hip", "noalloc", []), ("panel.hip", "panel", []),
           ("api.hip", "api", []), ("server.cpp", "server", []),
           ("linalg.cpp", "linalg_generic", ["-DLA_IMPL=la_generic"]),
           ("linalg.cpp", "linalg_v3", ["-DLA_IMPL=la_v3", "-march=x86-64-v3"]),
           ("linalg_dispatch.cpp", "linalg_dispatch", [])]
HOST_ONLY = ("linalg.cpp", "linalg_dispatch.cpp")
# every source that defines device code (hashed by bench.py to match counter records)
KERNEL_SOURCES = ["bmg_internal.h", "rowpass.h", "pass_f64.hip", "pass_f32.hip", "pass_bf16.hip",
                  "kernels.hip", "colpass.hip", "units.h", "rke.hip", "noalloc.hip", "panel.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions in the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def _compile(entry, objdir: str, verbose: bool) -> str:
    src, name, extra = entry
    obj = os.path.join(objdir, name + ".o")
    path = os.path.join(HERE, "csrc", src)
    host_flags = [f for f in FLAGS if not f.startswith("--offload")
                  and f not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
    if src in HOST_ONLY:       # plain host C++
        cmd = ["g++"] + host_flags + extra + ["-c", path, "-o", obj]
    elif src.endswith(".cpp"):  # host C++ calling the HIP runtime
        cmd = ["hipcc", "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + host_flags \
            + extra + ["-c", path, "-o", obj]
    else:
        cmd = ["hipcc"] + FLAGS + extra + ["-c", path, "-o", obj]
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
