"""Build libmfg.so (the HIP library behind include/mfg.h) for gfx950, in-tree.

Usage: python -m paper_2507_01958_amd.build   (or build() from Python).
Every call recompiles; objects go to paper_2507_01958_amd/_build/.

It also builds _build/asan/libmfg_host_asan.so: the same sources with the
host code instrumented by AddressSanitizer (the device code is not; -O1), for
the CPU tests of the C ABI's host paths (loaded with MFG_LIBRARY and the ASan
runtime preloaded; see tests/test_abi_asan.py).
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmfg.so")
SOURCES = ["api.hip", "stencil.hip", "vec.hip", "precond.hip", "tgemm.hip", "adjoint.hip",
           "batch.hip", "tune.hip", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=fast",
    # never emit packed fp32 arithmetic (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


ASAN_BUILD = os.path.join(BUILD, "asan")
ASAN_LIB = os.path.join(ASAN_BUILD, "libmfg_host_asan.so")
# host code only: each -fsanitize= goes to the host pass
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, asan: bool = False) -> str:
    out_dir = ASAN_BUILD if asan else BUILD
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    flags = [f if f != "-O3" else "-O1" for f in CFLAGS] + ASAN_FLAGS if asan else CFLAGS
    cmd = [HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def _link(objs, out, extra=()):
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False, asan: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(ASAN_BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = [(s, False) for s in srcs] + ([(s, True) for s in srcs] if asan else [])
    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(lambda j: _compile(*j), jobs))
    _link(objs[: len(srcs)], LIB)
    if asan:
        _link(objs[len(srcs):], ASAN_LIB, ASAN_FLAGS[:2])
    if verbose:
        print("built", LIB + (" and " + ASAN_LIB if asan else ""))
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
