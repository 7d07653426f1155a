"""GPU reverse sweep (mfg_cp_adjoint, torch.autograd) against the oracle's
reverse pass with exact projections, and against central finite differences of
the GPU forward.

Tolerance: normwise relative error of dJ/dm0 and dJ/dV <= 1e-7 against the
oracle (both sides solve to ~1e-12; the solve error enters the gradient
amplified by at most the condition of the reduced matrix on the forward and
reverse sweeps); <= 1e-5 against finite differences (truncation O(h^2) and
solve noise O(rtol/h)).
"""
import numpy as np
import pytest

from _gpu import dev, grid_of, host, say
from oracle import adjoint as oadj
from oracle import cp as ocp
from paper_2507_01958_amd import autograd as mad
from paper_2507_01958_amd import mfg
from paper_2507_01958_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _problem(inst):
    return mfg.make_problem(inst.d, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                            l=inst.l, T=inst.T, lo=inst.lo, hi=inst.hi)


@pytest.mark.parametrize("case", [(2, "periodic", 8, 6, 5), (2, "neumann", 12, 8, 6),
                                  (1, "periodic", 16, 1, 8)])
def test_adjoint_matches_oracle(case):
    import torch
    d, bc, nx, ny, nt = case
    inst = wl.small_instance(3, d, nx, ny, nt, bc, 0.1)
    g = grid_of(inst)
    mt = wl.gaussian_mixture(np.random.default_rng(9), d, nx, ny, bc, 3)
    iters = 13
    say(f"adjoint {case}")
    st, _ = ocp.cp_solve(g, inst.V, inst.m0, iters, method="direct")
    _, gy = oadj.terminal_loss_grad(g, st.y, mt)
    gm0_ref, gV_ref, _ = oadj.cp_gradient(g, inst.V, inst.m0, iters, gy)
    m0 = dev(inst.m0).requires_grad_(True)
    V = dev(inst.V).requires_grad_(True)
    y = mad.cp_solve(_problem(inst), m0, V, iters, rtol=1e-12, maxit=500, every=4)
    mT = mad.terminal_m(_problem(inst), y)
    loss = 0.5 * ((mT - dev(mt)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    for got, ref in [(host(m0.grad), gm0_ref), (host(V.grad), gV_ref)]:
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= 1e-7, err


def test_adjoint_matches_finite_differences_on_gpu():
    import torch
    inst = wl.small_instance(11, 2, 32, 32, 16, "periodic", 5e-2)
    mt = wl.gaussian_mixture(np.random.default_rng(12), 2, 32, 32, "periodic", 5)
    prob = _problem(inst)
    iters, rtol = 20, 1e-12
    say("adjoint vs FD 32x32x16")

    def loss_of(m0, V):
        y = mad.cp_solve(prob, m0, V, iters, rtol=rtol, maxit=800, every=10)
        return 0.5 * ((mad.terminal_m(prob, y) - dev(mt)) ** 2).sum()

    m0 = dev(inst.m0).requires_grad_(True)
    V = dev(inst.V).requires_grad_(True)
    loss_of(m0, V).backward()
    gm0, gV = host(m0.grad), host(V.grad)
    rng = np.random.default_rng(3)
    for which, grad in [("m0", gm0), ("V", gV)]:
        # m0 must stay non-negative: perturb it multiplicatively
        e = inst.m0 * rng.uniform(-1, 1, inst.M) if which == "m0" else rng.standard_normal(inst.M)
        base = inst.m0 if which == "m0" else inst.V
        h = 1e-5 * np.linalg.norm(base) / np.linalg.norm(e)
        with torch.no_grad():
            def J(x):
                m = dev(inst.m0 + (x * e if which == "m0" else 0.0))
                v = dev(inst.V + (x * e if which == "V" else 0.0))
                return float(loss_of(m, v))
            fd = (J(h) - J(-h)) / (2 * h)
        an = float(grad @ e)
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-12, (which, fd, an)
