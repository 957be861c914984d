"""Build the gfx950 shared library ``_lib/libsand.so`` from ``csrc/``.

Every HIP source is compiled with hipcc for gfx950 only, with packed FP32
instructions disabled, and linked into one shared library that exports the
C ABI of include/sand.h. Objects build in parallel; ``build()`` always
recompiles.
"""

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libsand.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# the kernel sources first (the forward ones take longest)
SOURCES = ["tmlp_sine.hip", "tmlp_finer.hip", "adjoint_sine.hip", "adjoint_finer.hip", "tmlp.hip",
           "adjoint.hip", "lookup.hip", "mapbuild.hip", "octree.hip", "api.cpp", "server.cpp",
           "noalloc.cpp"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument"]


def _compile(src):
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-I", SRC, "-c", os.path.join(SRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    return obj, err


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        results = list(ex.map(_compile, SOURCES))
    if verbose:
        for (_, err), src in zip(results, SOURCES):
            if err:
                print(f"[{src}]\n{err}", file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp,
           *[o for o, _ in results]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
