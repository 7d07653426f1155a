"""GPU check of mfg_pcg_noalloc, the PCG entry point that allocates no device
memory: through the C ABI, two calls in a row (the second on a smaller
problem, so it runs on what the first left in the shared scratch array) must
agree with mfg_pcg on a plan of the same problem, to the float64 parity bar:
the same iteration count, solutions equal to 1e-10 of their max norm, and the
true residual within the tolerance. A problem beyond the scratch limit is
rejected with MFG_ERR_UNSUPPORTED before any device work."""
import numpy as np
import pytest

from _gpu import dev, empty, host, plan_of, say
from paper_2507_01958_amd import mfg
from paper_2507_01958_amd import workloads as wl

pytestmark = pytest.mark.gpu

CASES = [
    # (d, nx, ny, nt, bc, nu, precision)
    (2, 64, 48, 32, "neumann", 0.02, "fp64"),
    (2, 16, 24, 12, "periodic", 0.1, "fp64"),
    (2, 128, 128, 64, "periodic", 0.01, "mixed_fp32"),
    (1, 36, 1, 20, "neumann", 0.1, "mixed_fp32"),
]


def _problem(inst, precision):
    return mfg.make_problem(inst.d, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                            l=inst.l, precision=precision, T=inst.T, lo=inst.lo, hi=inst.hi)


def _case(c, seed):
    d, nx, ny, nt, bc, nu, precision = c
    return wl.small_instance(700 + seed, d, nx, ny, nt, bc, nu), precision


@pytest.mark.parametrize("pair", [(0, 1), (2, 3)])
def test_noalloc_matches_pcg_on_consecutive_calls(pair):
    rtol = 1e-12
    for k, idx in enumerate(pair):
        inst, precision = _case(CASES[idx], idx)
        say(f"noalloc call {k + 1}: {inst.name} {precision}")
        b = dev(wl.random_vector(40 + idx, inst.n))
        u0 = empty(inst.n)
        with plan_of(inst, precision=precision) as P:
            its0, rel0, _ = mfg.mfg_pcg(P, b, u0, rtol, 400)
        u1 = empty(inst.n)
        u1.fill_(np.nan)  # the entry point must write every entry
        its1, rel1, rc = mfg.mfg_pcg_noalloc(_problem(inst, precision), b, u1, rtol, 400)
        a, r = host(u1), host(u0)
        assert rc == 0
        assert its1 == its0, (its1, its0)
        assert rel1 <= 2 * rtol and rel0 <= 2 * rtol
        assert np.abs(a - r).max() <= 1e-10 * np.abs(r).max()


def test_noalloc_rejects_too_large_and_long_horizon():
    import torch
    big = mfg.make_problem(2, 256, 256, 128, "neumann", 0.01, 5e-3)      # 2^23 cells
    b = torch.zeros(8, dtype=torch.float64, device="cuda")
    u = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(mfg.MFGError) as e:
        mfg.mfg_pcg_noalloc(big, b, u, 1e-8, 10)
    assert e.value.code == 2
    long = mfg.make_problem(1, 16, 1, 256, "periodic", 0.1, 5e-4)
    with pytest.raises(mfg.MFGError) as e:
        mfg.mfg_pcg_noalloc(long, b, u, 1e-8, 10)
    assert e.value.code == 2
