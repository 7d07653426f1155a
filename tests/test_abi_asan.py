"""The C ABI's host paths under AddressSanitizer (CPU, no GPU needed).

`paper_2507_01958_amd.build` also builds `_build/asan/libmfg_host_asan.so`,
the library with its host code instrumented. A child process preloads the ASan
runtime, loads that library through MFG_LIBRARY and drives the entry points'
argument checks, error reporting and problem validation (every error path that
returns before touching a device), including the per-axis boundary, q' and
batch arguments. It must exit cleanly with no AddressSanitizer report.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN_LIB = os.path.join(ROOT, "paper_2507_01958_amd", "_build", "asan", "libmfg_host_asan.so")


def _asan_runtime():
    cands = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return cands[-1] if cands else None


SCRIPT = r"""
import ctypes, sys
sys.path.insert(0, ROOT)
from paper_2507_01958_amd import mfg
lib = mfg.load()
assert b"gfx950" in lib.mfg_version()
h = ctypes.c_void_p()
def plan_rc(**kw):
    args = dict(d=2, nx=8, ny=8, nt=4, bc="periodic", nu=0.1, gamma=5e-4)
    args.update(kw)
    pb = mfg.make_problem(args.pop("d"), args.pop("nx"), args.pop("ny"), args.pop("nt"),
                          args.pop("bc"), args.pop("nu"), args.pop("gamma"), **args)
    rc = lib.mfg_plan(ctypes.byref(pb), None, None, None, ctypes.byref(h))
    msg = lib.mfg_last_error()
    assert isinstance(msg, bytes) and len(msg) > 0
    return rc
assert plan_rc(d=3) == 1
assert plan_rc(nx=10) == 2
assert plan_rc(nt=1) == 1
assert plan_rc(nu=-1.0) == 1
assert plan_rc(gamma=0.0) == 1
assert plan_rc(l=3) == 1
assert plan_rc(precision="fp64", coupling="linear", beta=-1.0) == 1
for qp in (1.0, 1.1, 8.0):
    assert plan_rc(qprime=qp) == 2
assert plan_rc(d=1, ny=1, bc=("periodic", "neumann")) == 1
assert plan_rc(bc=4) == 1
assert plan_rc(nx=1024, ny=1024, nt=2048) == 2
# NULL arguments
assert lib.mfg_plan(None, None, None, None, ctypes.byref(h)) == 1
assert lib.mfg_prox(None, None, 1.0, None) == 1
assert lib.mfg_destroy(None) == 0
assert lib.mfg_plan_batch(None, None, None, 0, None, None) == 1
for _ in range(1000):   # repeated error strings (thread-local buffer)
    plan_rc(d=3)
print("asan-clean")
"""


@pytest.mark.skipif(not os.path.exists(ASAN_LIB), reason="host-ASan library not built")
@pytest.mark.skipif(_asan_runtime() is None, reason="no ASan runtime")
def test_abi_host_paths_under_asan():
    env = dict(os.environ)
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = _asan_runtime() + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["MFG_LIBRARY"] = ASAN_LIB
    res = subprocess.run([sys.executable, "-c", f"ROOT = {ROOT!r}\n" + SCRIPT], env=env,
                         capture_output=True, text=True, timeout=300)
    assert "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    assert res.returncode == 0, (res.stdout[-2000:], res.stderr[-4000:])
    assert "asan-clean" in res.stdout
