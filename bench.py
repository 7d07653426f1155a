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

# Published MI355X peaks used for the roofline fraction.
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "fp16": 2500.0, "bf16": 2500.0}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_neumann256x256x128.json")
# the grid the stored counter readings were taken on (d, N_x, N_y, N_t, bc)
TRAFFIC_GRID = (2, 256, 256, 128, "neumann")


def kernel_sources_hash():
    """Hash of the HIP sources; stored HBM-counter readings are only reported
    while it matches (a changed kernel invalidates them)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2507_01958_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic(kernel, inst, variant, its=1.0, steps=1):
    """Algorithmic work of ONE launch of `kernel` on this workload (averaged
    over the launches of a `steps`-step CP call with `its` PCG iterations per
    solve where the launches differ): the minimal HBM bytes of a fused
    implementation, or the flops of the float64 time GEMM (matrix-core bound:
    2 N_t flops per element against 16 bytes)."""
    n = inst.n
    nb = 1 + 2 * inst.d  # primal blocks
    flex = variant in ("mixed_fp16", "mixed_bf16")  # PCG form with that preconditioner
    # the first update of a solve writes x without reading it; inside a call the
    # right-hand side reads z = xi + sigma ybar and the back-projection writes z
    # instead of xi and ybar, except on the call's first / last step
    upd = (6 * its - 1) / its
    rhs = ((steps - 1) * (nb + 1) + (2 * nb + 1)) / steps
    bp = ((steps - 1) * (1 + 3 * nb) + (1 + 4 * nb)) / steps
    if kernel.startswith("tgemm_f64"):
        return "mfma", 2.0 * inst.nt * inst.nt * inst.M, "fp64"
    # above N_t = 128 the low-precision transforms stream V and are priced on
    # the float16 / bfloat16 matrix cores (2 N_t flops per element against 12
    # or 16 bytes: about the ridge); the float32 mode is a two-term float16
    # split, three products per element pair
    if kernel.startswith("tgemm_") and inst.nt > 128:
        mult = 3.0 if kernel.startswith("tgemm_f32") else 1.0
        return "mfma", mult * 2.0 * inst.nt * inst.nt * inst.M, "fp16"
    for base in ("rows_fwd", "rows_inv", "rows_solve", "cols_solve"):
        if kernel in (base + "_f64", base + "_f32"):
            # one read and one write of the intermediate in the solve's precision
            return "hbm", 2 * (8 if kernel.endswith("f64") else 4) * n, None
    table = {
        "aat_fused": 4 * 8 * n,      # read z, p_old; write p_new, q
        "aat": 2 * 8 * n,
        "update": upd * 8 * n,       # read x, r, p, q; write x, r
        "pcg_init": 2 * 8 * n,       # read b; write r
        "residual": 2 * 8 * n,
        "rhs": rhs * 8 * n,          # read z (or xi, ybar); write r
        "backproj_prox": bp * 8 * n,  # read u, y; write y, z (or y, xi, ybar)
        "cp_init": 3 * nb * 8 * n,
        "adj_prox": (4 * nb + 1) * 8 * n,        # read gy, gybar, v, gxi; write gy, gxi, gV
    }
    if kernel.startswith("update_tgemm_rows_"):
        # the update and the forward preconditioner pass in one launch: the
        # update's bytes, then the float32 intermediate written
        return "hbm", upd * 8 * n + 4 * n, None
    if kernel.startswith("tgemm_") and kernel.endswith("_fwd"):
        return "hbm", (8 + 4) * n, None          # read r (f64), write f32
    if kernel.startswith(("tgemm_", "rows_tgemm_")) and kernel.endswith("_inv"):
        return "hbm", (4 + 8 + 8 + (8 if flex else 0)) * n, None  # + r (and q) for the dots
    if kernel in table:
        return "hbm", table[kernel], None
    return None, None, None


def roofline(report, inst, variant, its, steps):
    """Roofline object of the dominant kernel (largest total time)."""
    cands = {k: v for k, v in report.items() if k != "finish"}
    dom = max(cands, key=lambda k: cands[k]["total_ms"])
    calls = cands[dom]["calls"]
    avg_s = cands[dom]["total_ms"] / 1e3 / calls
    bound, work, dtype = algorithmic(dom, inst, variant, its, steps)
    out = {"kernel": dom, "bound": bound, "calls": calls, "avg_us": avg_s * 1e6}
    if bound == "mfma":
        out.update(achieved=work / avg_s / 1e12, peak=PEAK_TFLOPS[dtype], unit="TFLOP/s",
                   algorithmic_per_launch=work)
    elif bound == "hbm":
        out.update(achieved=work / avg_s / 1e9, peak=PEAK_HBM_GBS, unit="GB/s",
                   algorithmic_per_launch=work)
    if bound:
        out["frac"] = out["achieved"] / out["peak"]
    out["traffic"] = None
    try:
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        kern = tr.get("variants", {}).get(variant, {})
        same_grid = (inst.d, inst.nx, inst.ny, inst.nt, inst.bc) == TRAFFIC_GRID
        if same_grid and tr.get("sources_hash") == kernel_sources_hash() and dom in kern:
            out["traffic"] = kern[dom]["bytes_per_launch"]
    except (OSError, ValueError):
        pass
    return out


def cpu_baseline(inst, seconds_hint=12.0):
    """The oracle as it stands (fast mode: PCG with Algorithms 1+2 through a
    dense V and scipy.fft) timed on the host: CP iterations from the initial
    point at the same PCG tolerance, on a bounded sample."""
    import threadpoolctl
    from oracle import cp as ocp
    from oracle import operators as ops
    from oracle.grid import Grid
    g = Grid(d=inst.d, nx=inst.nx, ny=inst.ny, nt=inst.nt, bc=inst.bc, nu=inst.nu, T=inst.T,
             l=1, gamma=inst.gamma)
    t0 = time.perf_counter()
    S = ops.Spatial(g)
    setup = time.perf_counter() - t0
    st = ocp.cp_init(g, inst.m0)
    proj = ocp.Projector(g, S, "pcg", RTOL, PCG_MAXIT)
    iters, t_iter = 0, 0.0
    # whole CP iterations until about seconds_hint of work (at most 8)
    while iters < 8 and t_iter < seconds_hint:
        t1 = time.perf_counter()
        ocp.cp_step(g, S, st, inst.V, inst.m0, proj)
        t_iter += time.perf_counter() - t1
        iters += 1
    threads = 1
    for info in threadpoolctl.threadpool_info():
        threads = max(threads, int(info.get("num_threads", 1)))
    return {"value": iters / t_iter, "unit": "CP iters/s", "cores": threads, "kind": "oracle",
            "sample": f"{iters} CP iterations of the float64 oracle (PCG with Algorithms 1+2 via "
                      f"dense V and scipy.fft, rtol {RTOL:g}) on the same 256x256x128 workload; "
                      f"setup {setup:.1f} s excluded; {os.cpu_count()} host CPUs visible"}


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
    ap.add_argument("--workload", default="neumann256",
                    choices=["neumann256", "batch", "grad", "adaptive", "paper", "torus1d",
                             "nu_sweep"],
                    help="neumann256: the headline line; batch: 32 uneven periodic instances, "
                         "batched vs one plan at a time; grad: gradient through 50 CP "
                         "iterations; adaptive: time to solution with the Section 5 "
                         "stopping and inner-tolerance rules; paper: the paper's Problems 1 "
                         "and 2 at N_x = 64, N_t = 512 with those rules; torus1d: 200 CP "
                         "iterations on the 1-D torus 64x32 at rtol 1e-10; nu_sweep: 500 CP "
                         "iterations on the 2-D torus 128^2x64 for four nu, FP64 vs FP32")
    ap.add_argument("--cp-iters", type=int, default=0,
                    help="CP iterations of the torus1d / nu_sweep runs (0: 200 / 500)")
    ap.add_argument("--batch", type=int, default=32, help="instances of the batch workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of tuning them first")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device copy (HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy():
    """A plain device-to-device copy of known size (512 MiB read + 512 MiB
    written), repeated 4 times; used to scale the HBM byte counters."""
    import torch
    n = (512 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n,
                      "repeats": 4}))


def _problem(inst, precision):
    from paper_2507_01958_amd import mfg
    return mfg.make_problem(inst.d, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                            l=inst.l, precision=precision, T=inst.T, lo=inst.lo, hi=inst.hi)


def bench_batch(args):
    """Uneven batch of independent periodic problems (sizes 64^2..256^2, N_t 32..128,
    nu log-uniform in [1e-3, 1]): instance-CP-iterations per second of the
    batched path (one launch per phase over all instances, steps replayed from a
    HIP graph) against running the same instances one plan at a time."""
    import numpy as np
    import torch

    from paper_2507_01958_amd import mfg
    from paper_2507_01958_amd import workloads as wl

    insts = [wl.batch_instance(i) for i in range(args.batch)]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    Vs = [torch.from_numpy(i.V).to(dev) for i in insts]
    m0s = [torch.from_numpy(i.m0).to(dev) for i in insts]
    prec = "mixed_fp32"
    batched = {}
    for variant in (prec, "fp64"):
        B = mfg.mfg_plan_batch([_problem(i, variant) for i in insts], Vs, m0s, stream)
        if not args.no_autotune:
            mfg.mfg_batch_autotune(B, 1)
        states = [mfg.CPState(p) for p in B.plans]
        for p, st in zip(B.plans, states):
            mfg.mfg_cp_init(p, st)
        mfg.mfg_batch_cp_solve(B, states, args.warmup, RTOL, PCG_MAXIT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its_v = mfg.mfg_batch_cp_solve(B, states, args.steps, RTOL, PCG_MAXIT)
        torch.cuda.synchronize()
        dt_v = time.perf_counter() - t0
        B.close()
        del states
        batched[variant] = len(insts) * args.steps / dt_v
        if variant == prec:
            its, dt_batch = its_v, dt_v
    rate_batch = batched[prec]
    seq = {}
    for variant in ("fp64", prec):
        total = 0.0
        for inst, V, m0 in zip(insts, Vs, m0s):
            P = mfg.mfg_plan(_problem(inst, variant), V, m0, stream)
            if not args.no_autotune:
                mfg.mfg_autotune(P, 1)
            st = mfg.CPState(P)
            mfg.mfg_cp_init(P, st)
            mfg.mfg_cp_solve(P, st, args.warmup, RTOL, PCG_MAXIT, stats=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mfg.mfg_cp_solve(P, st, args.steps, RTOL, PCG_MAXIT, stats=False)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
            P.close()
        seq[variant] = len(insts) * args.steps / total
    n_total = sum(i.n for i in insts)
    out = {
        "metric": "instance CP iters/s, batch of independent 2D periodic problems",
        "value": rate_batch,
        "unit": "instance CP iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt_batch / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+fp32", "data": "synthetic (seeded)",
        "config": {"workload": f"batch{len(insts)}_periodic_uneven", "pcg_rtol": RTOL,
                   "instances": [i.name for i in insts], "sum_n": n_total,
                   "variant": prec},
        "batched_instance_cp_iters_per_s": batched,
        "sequential_instance_cp_iters_per_s": seq,
        "speedup_vs_sequential": {k: rate_batch / v for k, v in seq.items()},
        "speedup_same_precision": {k: batched[k] / seq[k] for k in batched},
        "mean_pcg_iters": float(np.mean(its)), "max_pcg_iters": int(np.max(its)),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def bench_grad(args):
    """dJ/dm0 and dJ/dV of J = 1/2 ||m(., T) - m_target||^2 through 50 CP
    iterations (PCG rtol 1e-10, checkpoint every 10) on the 2-D torus 256^2 x 100,
    nu = 5e-2: gradient evaluations (forward + reverse sweep) per second."""
    import torch

    from paper_2507_01958_amd import autograd as mad
    from paper_2507_01958_amd import workloads as wl

    inst, mt = wl.gradient_instance()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pb = _problem(inst, "fp64")
    target = torch.from_numpy(mt).to(dev)
    n_iter, every, rtol = 50, 10, 1e-10
    fwd, bwd = [], []
    for rep in range(args.warmup + args.steps):
        m0 = torch.from_numpy(inst.m0).to(dev).requires_grad_(True)
        V = torch.from_numpy(inst.V).to(dev).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = mad.cp_solve(pb, m0, V, n_iter, rtol=rtol, maxit=1000, every=every)
        J = 0.5 * ((mad.terminal_m(pb, y) - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep >= args.warmup:
            fwd.append(t1 - t0)
            bwd.append(t2 - t1)
    tot = sum(fwd) + sum(bwd)
    out = {
        "metric": "gradient evaluations/s through 50 CP iterations (d=2 periodic 256^2x100)",
        "value": args.steps / tot,
        "unit": "gradients/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * tot / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded)",
        "config": {"workload": f"grad_periodic{inst.nx}x{inst.ny}x{inst.nt}_nu{inst.nu:g}",
                   "cp_iters": n_iter, "checkpoint_every": every, "pcg_rtol": rtol},
        "forward_ms": 1e3 * sum(fwd) / args.steps, "reverse_ms": 1e3 * sum(bwd) / args.steps,
        "J": float(J.detach().cpu()),
        "grad_norms": {"m0": float(m0.grad.norm().cpu()), "V": float(V.grad.norm().cpu())},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def bench_adaptive(args):
    """Time to solution on the 256^2 x 128 Neumann workload with the Section 5
    rules: CP until ||m_{l+1} - m_l|| <= 1e-4 ||m0||, each projection by PCG to
    min(1e-4, max(1e-6, 1e-4 r)), from the initial point; FP64 and the FP32
    preconditioner, the latter also with each PCG started from the previous
    projection's solution. `steps` solves are timed after `warmup` untimed ones."""
    import numpy as np
    import torch

    from paper_2507_01958_amd import mfg
    from paper_2507_01958_amd import workloads as wl

    inst = wl.neumann_square(n=args.size, nt=args.nt)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    V = torch.from_numpy(inst.V).to(dev)
    m0 = torch.from_numpy(inst.m0).to(dev)
    cp_tol = 1e-4 * float(np.linalg.norm(inst.m0))
    res = {}
    for name in ["fp64", "mixed_fp32", "mixed_fp32_warm"]:
        variant = name.replace("_warm", "")
        with mfg.mfg_plan(_problem(inst, variant), V, m0) as P:
            if not args.no_autotune:
                mfg.mfg_autotune(P, 1)
            mfg.mfg_set_warm_start(P, name.endswith("_warm"))
            st = mfg.CPState(P)
            times = []
            for rep in range(args.warmup + args.steps):
                mfg.mfg_cp_init(P, st)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = mfg.mfg_cp_solve_tol(P, st, 5000, cp_tol, 1000)
                torch.cuda.synchronize()
                if rep >= args.warmup:
                    times.append(time.perf_counter() - t0)
            t = sum(times) / len(times)
            res[name] = {"seconds": t, "cp_iters": out["n_done"],
                            "pcg_iters_total": int(sum(out["pcg_iters"])),
                            "final_dm": out["dm"][-1], "cp_iters_per_s": out["n_done"] / t}
    best = min(res, key=lambda k: res[k]["seconds"])
    print(json.dumps({
        "metric": "time to solution, CP to ||dm|| <= 1e-4 ||m0|| with the CGtol rule (2D 256^2x128)",
        "value": res[best]["seconds"], "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * res[best]["seconds"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else "f64+fp32", "data": "synthetic (seeded)",
        "config": {"workload": f"neumann2d_{inst.nx}x{inst.ny}x{inst.nt}_nu{inst.nu:g}_adaptive",
                   "cp_tol": cp_tol, "variant": best},
        "variants": res, "roofline": None, "cpu_baseline": None,
    }))


def _run_fixed(inst, variant, n_iter, rtol, warmup_runs=1):
    """n_iter CP iterations from the initial point at PCG tolerance rtol, timed
    after `warmup_runs` untimed identical runs; returns (seconds, stats, state)."""
    import torch

    from paper_2507_01958_amd import mfg
    dev = torch.device("cuda:0")
    V = torch.from_numpy(inst.V).to(dev)
    m0 = torch.from_numpy(inst.m0).to(dev)
    P = mfg.mfg_plan(_problem(inst, variant), V, m0)
    st = mfg.CPState(P)
    for rep in range(warmup_runs + 1):
        mfg.mfg_cp_init(P, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = mfg.mfg_cp_solve(P, st, n_iter, rtol, 1000)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
    y = st.y.clone()
    xi = st.xi.clone()
    P.close()
    return t, stats, y, xi


def bench_torus1d(args):
    """The 1-D torus workload (N_x = 64, N_t = 32, nu = 0.1, V = sin(2 pi x)/2,
    three Gaussian bumps): 200 CP iterations with PCG to rtol 1e-10, FP64 and the
    FP32 preconditioner; CP iterations per second of the whole run."""
    import numpy as np
    import torch

    from paper_2507_01958_amd import workloads as wl
    torch.cuda.set_device(0)
    inst = wl.torus_1d()
    n_iter = args.cp_iters or 200
    res = {}
    for variant in ("fp64", "mixed_fp32"):
        t, stats, y, xi = _run_fixed(inst, variant, n_iter, 1e-10, args.warmup and 1)
        res[variant] = {"seconds": t, "cp_iters_per_s": n_iter / t,
                        "mean_pcg_iters": float(np.mean(stats["pcg_iters"])), "y": y}
    ref = res["fp64"].pop("y")
    dev = (res["mixed_fp32"].pop("y") - ref).abs().max().item() / ref.abs().max().item()
    res["mixed_fp32"]["deviation_vs_fp64"] = dev
    print(json.dumps({
        "metric": "CP iters/s, 1-D torus 64x32, 200 CP iterations at PCG rtol 1e-10",
        "value": res["fp64"]["cp_iters_per_s"], "unit": "CP iters/s",
        "n_gpus": 1, "steps": n_iter, "warmup": 1,
        "ms_per_step": 1e3 * res["fp64"]["seconds"] / n_iter,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded)",
        "config": {"workload": f"torus1d_{inst.nx}x{inst.nt}_nu{inst.nu:g}", "pcg_rtol": 1e-10,
                   "cp_iters": n_iter},
        "variants": res, "roofline": None, "cpu_baseline": None,
    }))


def bench_nu_sweep(args):
    """The 2-D torus 128^2 x 64 with V = sin(2 pi x) cos(2 pi y) over
    nu in {1e-3, 1e-2, 1e-1, 1}: 500 CP iterations with PCG to rtol 1e-8, FP64
    against the FP32 preconditioner; CP iterations per second, mean PCG
    iterations, and the deviation of the mixed run's final iterate (max-norm,
    relative, per block: m, w, and the multiplier xi)."""
    import numpy as np
    import torch

    from paper_2507_01958_amd import workloads as wl
    torch.cuda.set_device(0)
    n_iter = args.cp_iters or 500
    res = {}
    tot = {"fp64": [0, 0.0], "mixed_fp32": [0, 0.0]}
    for nu in (1e-3, 1e-2, 1e-1, 1.0):
        inst = wl.torus_2d_trig(nu=nu)
        r = {}
        for variant in ("fp64", "mixed_fp32"):
            t, stats, y, xi = _run_fixed(inst, variant, n_iter, RTOL, args.warmup and 1)
            r[variant] = {"seconds": t, "cp_iters_per_s": n_iter / t,
                          "mean_pcg_iters": float(np.mean(stats["pcg_iters"])),
                          "_y": y, "_xi": xi}
            tot[variant][0] += n_iter
            tot[variant][1] += t
        n = inst.n
        a, b = r["mixed_fp32"], r["fp64"]
        rel = lambda u, v: (u - v).abs().max().item() / max(v.abs().max().item(), 1e-300)
        a["deviation_vs_fp64"] = {"m": rel(a["_y"][:n], b["_y"][:n]),
                                  "w": rel(a["_y"][n:], b["_y"][n:]),
                                  "xi": rel(a["_xi"], b["_xi"])}
        for v in r.values():
            v.pop("_y")
            v.pop("_xi")
        res[f"nu={nu:g}"] = r
    rates = {k: c / t for k, (c, t) in tot.items()}
    best = max(rates, key=rates.get)
    print(json.dumps({
        "metric": "CP iters/s over the nu sweep, 2-D torus 128^2x64, 500 CP iterations, "
                  "PCG rtol 1e-8",
        "value": rates[best], "unit": "CP iters/s",
        "n_gpus": 1, "steps": 4 * n_iter, "warmup": 1,
        "ms_per_step": 1e3 / rates[best],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else "f64+fp32", "data": "synthetic (seeded)",
        "config": {"workload": "torus2d_128x128x64_nu_sweep", "pcg_rtol": RTOL,
                   "cp_iters_per_nu": n_iter, "variant": best},
        "sweep_cp_iters_per_s": rates, "per_nu": res, "roofline": None, "cpu_baseline": None,
    }))


# The paper's own runs at N_x = 64, N_t = 512, nu = 1e-2 (Tables 5.1 and 5.3, the
# DCT-VIII preconditioner, 32 CPU cores): CP iterations, average CG iterations
# per projection and total seconds. Context, not a target: another machine and a
# CPU implementation.
PAPER_CONTEXT = {"problem1": {"cp_iters": 70, "avg_cg": 2.4, "seconds": 234.78,
                              "table": "5.1"},
                 "problem2": {"cp_iters": 532, "avg_cg": 3.6, "seconds": 641.61,
                              "table": "5.3"}}


def bench_paper(args):
    """The paper's two problems (Section 5.1: periodic, f = m^2/2 + V with the
    trigonometric V, m0 = 1; Section 5.2: Neumann on [-1/2, 1/2]^2, f = 0, terminal
    cost (m - mbar)/beta with beta = 1e-3, Gaussian m0 and mbar) at the shape of
    Tables 5.1 / 5.3, N_x = N_y = 64, N_t = 8 N_x = 512, nu = 1e-2, solved with the
    Section 5 rules (CP until ||dm|| <= 1e-4 ||m0||, CGtol rule), FP64 and the FP32
    preconditioner; time to solution after one untimed solve."""
    import numpy as np
    import torch

    from paper_2507_01958_amd import mfg
    from paper_2507_01958_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, nt, nu = args.size if args.size != 256 else 64, args.nt if args.nt != 128 else 512, 1e-2
    res = {}
    for prob in ("problem1", "problem2"):
        if prob == "problem1":
            inst, coupling, beta, mbar = wl.paper_problem1(n, nt, nu), "quadratic", 0.0, None
        else:
            inst, mbar, beta = wl.paper_problem2(n, nt, nu)
            coupling = "potential"
        V = torch.from_numpy(inst.V).to(dev)
        m0 = torch.from_numpy(inst.m0).to(dev)
        cp_tol = 1e-4 * float(np.linalg.norm(inst.m0))
        res[prob] = {"paper": PAPER_CONTEXT[prob]}
        for variant in ("fp64", "mixed_fp32"):
            pb = mfg.make_problem(2, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma,
                                  l=1, precision=variant, T=inst.T, lo=inst.lo, hi=inst.hi,
                                  coupling=coupling, beta=beta)
            with mfg.mfg_plan(pb, V, m0) as P:
                if mbar is not None:
                    mfg.mfg_set_target(P, torch.from_numpy(mbar).to(dev))
                if not args.no_autotune:
                    mfg.mfg_autotune(P, 1)
                st = mfg.CPState(P)
                for rep in range(2):
                    mfg.mfg_cp_init(P, st)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    out = mfg.mfg_cp_solve_tol(P, st, 6000, cp_tol, 1000)
                    torch.cuda.synchronize()
                    t = time.perf_counter() - t0
            k = out["n_done"]
            res[prob][variant] = {"seconds": t, "cp_iters": k,
                                  "avg_pcg_iters": float(np.mean(out["pcg_iters"])),
                                  "converged": out["dm"][-1] <= cp_tol, "final_dm": out["dm"][-1],
                                  "cp_iters_per_s": k / t}
    best = min(("fp64", "mixed_fp32"), key=lambda v: res["problem1"][v]["seconds"])
    print(json.dumps({
        "metric": "time to solution of the paper's Problem 1 (64^2x512, nu=1e-2, Section 5 rules)",
        "value": res["problem1"][best]["seconds"], "unit": "s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * res["problem1"][best]["seconds"] / res["problem1"][best]["cp_iters"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+fp32" if best == "mixed_fp32" else "f64", "data": "analytic (Section 5)",
        "config": {"workload": f"paper_problems_{n}x{n}x{nt}_nu{nu:g}", "variant": best},
        "problems": res, "roofline": None, "cpu_baseline": None,
    }))


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "grad":
        bench_grad(args)
        return
    if args.workload == "adaptive":
        bench_adaptive(args)
        return
    if args.workload == "paper":
        bench_paper(args)
        return
    if args.workload == "torus1d":
        bench_torus1d(args)
        return
    if args.workload == "nu_sweep":
        bench_nu_sweep(args)
        return
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

    # the right-hand side of CP iteration 50 of the float64 run (the PCG
    # solves/s are measured on it, on the first one, and on a N(0,1) vector;
    # --pcg-reps 0 leaves the PCG solves out, e.g. for counter runs)
    b50 = None
    if args.pcg_reps > 0:
        with mfg.mfg_plan(_problem(inst, "fp64"), V, m0, stream) as P:
            st = mfg.CPState(P)
            mfg.mfg_cp_init(P, st)
            mfg.mfg_cp_solve(P, st, 49, RTOL, PCG_MAXIT, stats=False)
            z = st.xi + st.sigma * st.ybar
            b50 = torch.empty(inst.n, dtype=torch.float64, device=dev)
            mfg.mfg_apply_C(P, z, b50)
            b50[: inst.M] -= st.sigma * m0 * (inst.nt / inst.T)
            torch.cuda.synchronize()
            del st, z

    results = {}
    for variant in args.variants.split(","):
        pb = mfg.make_problem(2, inst.nx, inst.ny, inst.nt, inst.bc, inst.nu, inst.gamma, l=1,
                              precision=variant)
        P = mfg.mfg_plan(pb, V, m0, stream)
        if not args.no_autotune:
            mfg.mfg_autotune(P, 1)  # launch shapes for this workload (setup, not timed)
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
        # PCG solves: seeded N(0,1) right-hand side, the first projection's
        # right-hand side Cr ybar0 - dr (ybar0 = (m0 at every slice, w = 0)) and
        # the one of CP iteration 50 (from the float64 run above).
        rhs = {}
        rhs["randn"] = torch.from_numpy(wl.random_vector(33, inst.n)).to(dev)
        y0 = torch.zeros(P.nprimal, dtype=torch.float64, device=dev)
        y0[: inst.n] = m0.repeat(inst.nt)
        b1 = torch.empty(inst.n, dtype=torch.float64, device=dev)
        mfg.mfg_apply_C(P, y0, b1)
        b1[: inst.M] -= m0 * (inst.nt / inst.T)
        rhs["cp_iter1"] = b1
        rhs["cp_iter50"] = b50
        u = torch.empty(inst.n, dtype=torch.float64, device=dev)
        pcg = {}
        for name, b in (rhs.items() if args.pcg_reps > 0 else ()):
            its, rel, _ = mfg.mfg_pcg(P, b, u, RTOL, PCG_MAXIT, true_residual=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.pcg_reps):
                mfg.mfg_pcg(P, b, u, RTOL, PCG_MAXIT, true_residual=False)
            torch.cuda.synchronize()
            pt = (time.perf_counter() - t0) / args.pcg_reps
            pcg[name] = dict(solves_per_s=1.0 / pt, iters=its, true_relres=rel)
        # second pass with per-kernel HIP events on the plan's stream
        mfg.mfg_profile(P, True)
        mfg.mfg_cp_solve(P, st, args.steps, RTOL, PCG_MAXIT, stats=False)
        report = mfg.mfg_profile_report(P)
        mfg.mfg_profile(P, False)
        results[variant] = dict(cp_iters_per_s=cp_rate, ms_per_cp_iter=1e3 * dt / args.steps,
                                mean_pcg_iters=float(np.mean(stats["pcg_iters"])),
                                max_pcg_iters=int(np.max(stats["pcg_iters"])),
                                pcg=pcg,
                                roofline=roofline(report, inst, variant,
                                                  float(np.mean(stats["pcg_iters"])), args.steps),
                                kernels_us={k: round(1e3 * v["total_ms"] / v["calls"], 2)
                                            for k, v in report.items()})
        P.close()

    best = max(results, key=lambda k: results[k]["cp_iters_per_s"])
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inst)
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
        "pcg_solves_per_s": results[best]["pcg"].get("cp_iter1", {}).get("solves_per_s"),
        "roofline": results[best]["roofline"],
        "cpu_baseline": cpu,
        "variants": results,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
