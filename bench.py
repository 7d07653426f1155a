"""Throughput of the Chambolle-Pock / PCG hot path on one MI355X.

Workload: the 2-D Neumann unit square, 256 x 256 nodes, N_t = 128 (n = 8,388,608
unknowns in the reduced system, 41.9M primal unknowns), nu = 1e-2, f = m + V
with V a seeded random field of 8 cosine modes and m0 a seeded 5-bump Gaussian
mixture (synthetic, seed 3). One step = one accelerated Chambolle-Pock
iteration: right-hand side, PCG projection to a 1e-8 relative residual from a
zero initial guess, back-projection + prox + extrapolation.

Prints ONE JSON line (rank 0). `value` is CP iterations per second of the
fastest precision variant whose PCG reaches the same float64 residual; every
variant's CP iters/s and PCG solves/s are listed under `variants`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

RTOL = 1e-8
PCG_MAXIT = 200


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variants", default="fp64,mixed_fp32,mixed_fp16,mixed_bf16")
    ap.add_argument("--pcg-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--nt", type=int, default=128)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2507_01958_amd import mfg
    from paper_2507_01958_amd import workloads as wl

    inst = wl.neumann_square(n=args.size, nt=args.nt)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    V = torch.from_numpy(inst.V).to(dev)
    m0 = torch.from_numpy(inst.m0).to(dev)
    stream = torch.cuda.current_stream()

    results = {}
    for variant in args.variants.split(","):
        pb = mfg.make_problem(2, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma, l=1,
                              precision=variant)
        P = mfg.mfg_plan(pb, V, m0, stream)
        st = mfg.CPState(P)
        mfg.mfg_cp_init(P, st)
        # warmup
        mfg.mfg_cp_solve(P, st, args.warmup, RTOL, PCG_MAXIT, stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = mfg.mfg_cp_solve(P, st, args.steps, RTOL, PCG_MAXIT, stats=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cp_rate = args.steps / dt
        # PCG solves: seeded N(0,1) right-hand side and the first projection's
        # right-hand side Cr ybar0 - dr (ybar0 = (m0 at every slice, w = 0)).
        rhs = {}
        rhs["randn"] = torch.from_numpy(wl.random_vector(33, inst.n)).to(dev)
        y0 = torch.zeros(P.nprimal, dtype=torch.float64, device=dev)
        y0[: inst.n] = m0.repeat(inst.nt)
        b1 = torch.empty(inst.n, dtype=torch.float64, device=dev)
        mfg.mfg_apply_C(P, y0, b1)
        b1[: inst.M] -= m0 * (inst.nt / inst.T)
        rhs["cp_iter1"] = b1
        u = torch.empty(inst.n, dtype=torch.float64, device=dev)
        pcg = {}
        for name, b in rhs.items():
            its, rel, _ = mfg.mfg_pcg(P, b, u, RTOL, PCG_MAXIT, true_residual=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.pcg_reps):
                mfg.mfg_pcg(P, b, u, RTOL, PCG_MAXIT, true_residual=False)
            torch.cuda.synchronize()
            pt = (time.perf_counter() - t0) / args.pcg_reps
            pcg[name] = dict(solves_per_s=1.0 / pt, iters=its, true_relres=rel)
        results[variant] = dict(cp_iters_per_s=cp_rate, ms_per_cp_iter=1e3 * dt / args.steps,
                                mean_pcg_iters=float(np.mean(stats["pcg_iters"])),
                                max_pcg_iters=int(np.max(stats["pcg_iters"])),
                                pcg=pcg)
        P.close()

    best = max(results, key=lambda k: results[k]["cp_iters_per_s"])
    out = {
        "metric": "CP iters/s & PCG solves/s (1e-8 rel) at 2D 256^2x128; mixed vs FP64 GPU",
        "value": results[best]["cp_iters_per_s"],
        "unit": "CP iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[best]["ms_per_cp_iter"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else f"f64+{best.split('_')[1]}",
        "data": "synthetic (seeded)",
        "config": {"workload": f"neumann2d_{inst.nx}x{inst.ny}x{inst.nt}_nu{inst.nu:g}",
                   "pcg_rtol": RTOL, "variant": best, "l": 1},
        "variants": results,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
