"""Host-side checks of bench.py: the one-GPU contract and the cost model the
roofline uses (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2507_01958_amd import workloads as wl  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cost_model_bounds():
    inst = wl.neumann_square()
    n = inst.n
    assert bench.algorithmic("update", inst, "mixed_fp32", its=8) == ("hbm", (6 * 8 - 1) / 8 * 8 * n,
                                                                        None)
    assert bench.algorithmic("aat_fused", inst, "fp64")[:2] == ("hbm", 32 * n)
    bound, work, dtype = bench.algorithmic("tgemm_f64_fwd", inst, "fp64")
    assert (bound, dtype) == ("mfma", "fp64") and work == 2.0 * inst.nt * n
    # the low-precision GEMMs stream their operands at N_t <= 128 ...
    assert bench.algorithmic("tgemm_f32_fwd", inst, "mixed_fp32")[0] == "hbm"
    # ... and above it are priced on the float16 matrix cores (three products
    # per element pair for the float32 split)
    long = wl.neumann_square(n=64, nt=2048)
    bound, work, dtype = bench.algorithmic("tgemm_f32_inv", long, "mixed_fp32")
    assert (bound, dtype) == ("mfma", "fp16") and work == 3 * 2.0 * long.nt * long.n
    bound, work, dtype = bench.algorithmic("tgemm_f16_fwd", long, "mixed_fp16")
    assert (bound, dtype) == ("mfma", "fp16") and work == 2.0 * long.nt * long.n


@pytest.mark.parametrize("kernel", ["rows_fwd_f32", "cols_solve_f64", "rhs", "backproj_prox"])
def test_cost_model_covers_the_path(kernel):
    bound, work, _ = bench.algorithmic(kernel, wl.neumann_square(), "mixed_fp32", its=8, steps=20)
    assert bound == "hbm" and work > 0
