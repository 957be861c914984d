"""Host code under sanitizers, on the CPU (no GPU needed).

* The serving loop's scheduling pieces (paper_2604_25936_amd/csrc/batching.h:
  first-fit arena, FIFO admission, batch selection), unit-tested by
  tests/host/test_batching.cpp, built with g++ under AddressSanitizer +
  UndefinedBehaviorSanitizer and under ThreadSanitizer (the threaded part
  runs submitters, a scheduler and completers as the loop does).
* The library's host code (api.cpp, server.cpp) rebuilt with
  AddressSanitizer + UndefinedBehaviorSanitizer on the host side only and
  linked with the regular kernel objects; tests/test_abi.py then runs
  against that build (argument and blob validation, symbol exports,
  workspace sizes, server argument errors).
"""

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_25936_amd", "csrc")
LIBDIR = os.path.join(ROOT, "paper_2604_25936_amd", "_lib")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n--- stdout\n{r.stdout[-4000:]}\n--- stderr\n{r.stderr[-4000:]}"
    return r


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_batching_under_sanitizer(san, tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "test_batching")
    _run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={san}",
          "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(ROOT, "tests", "host",
                                                                 "test_batching.cpp"),
          "-o", exe, "-pthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = _run([exe], env=env)
    assert "batching tests passed" in r.stdout


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_abi_under_asan_ubsan(tmp_path):
    rt = _asan_runtime()
    objs = [os.path.join(LIBDIR, f) for f in
            ("tmlp_sine.o", "tmlp_finer.o", "adjoint_sine.o", "adjoint_finer.o", "tmlp.o",
             "adjoint.o", "lookup.o", "mapbuild.o", "octree.o")]
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("hipcc or the clang AddressSanitizer runtime not available")
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("kernel objects not built (run __graft_entry__.build())")
    flags = ["-x", "hip", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC",
             "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-I", CSRC]
    host = []
    procs = []
    for src in ("api.cpp", "server.cpp", "noalloc.cpp"):
        o = str(tmp_path / (src + ".o"))
        host.append(o)
        procs.append(subprocess.Popen([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, err[-4000:]
    lib = str(tmp_path / "libsand_asan.so")
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-shared-libsan",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-o", lib, *host, *objs])
    env = dict(os.environ, LD_PRELOAD=rt, SAND_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = _run([sys.executable, "-m", "pytest", "-q", "-s", "-p", "no:cacheprovider",
              os.path.join(ROOT, "tests", "test_abi.py")], env=env)
    assert " passed" in r.stdout and "failed" not in r.stdout
