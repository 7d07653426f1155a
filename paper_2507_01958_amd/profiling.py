"""Summaries of rocprofv3 databases for the library's kernels.

  python -m paper_2507_01958_amd.profiling stats DB --cmd "..." --out FILE.md
      per-kernel calls / average / total time from a --kernel-trace --stats run
  python -m paper_2507_01958_amd.profiling traffic --variant V --fetch DB --write DB \
         --cal-fetch DB --cal-write DB --out FILE.json [--merge]
      HBM bytes per launch from FETCH_SIZE / WRITE_SIZE passes, each scaled by
      what the same counter reads for a plain device copy of known size
  python -m paper_2507_01958_amd.profiling counters DB --variant V \
         --counters MfmaUtil MfmaFlops [--active MfmaFlops] --out FILE.json [--merge]
      per-kernel averages of counters from a --pmc run (rows of one dispatch
      summed), e.g. matrix-core busy percentage and matrix-core flops

Kernels are reported under the names the library's own profiler uses
(tgemm_f64_fwd, aat_fused, cols_solve, ...): a dispatch of a template kernel
is classified by its template arguments and, where one kernel serves two
roles (the float64 time GEMM, the row transforms), by its neighbours in the
dispatch order.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import re
import sqlite3
import sys

MODES = {"0": "f64", "1": "f32", "2": "f16", "3": "bf16"}


def _short(name: str) -> str:
    m = re.match(r"(?:void )?mfg::\(anonymous namespace\)::([^(]+)", name)
    return m.group(1).strip() if m else name


def _targs(s: str):
    """Template arguments of a short kernel name, as stripped strings."""
    if "<" not in s:
        return []
    return [a.strip() for a in s[s.index("<") + 1:s.rindex(">")].split(",")]


def _prec_sfx(s: str) -> str:
    return "_f64" if "double" in _targs(s)[:1] else "_f32"


def classify(seq):
    """Map an ordered list of raw kernel names to logical names."""
    shorts = [_short(n) for n in seq]
    out = []
    is_rows = lambda x: x.startswith("k_rows") and not x.startswith("k_rows_batch") \
        and not x.startswith("k_rows_reg_batch")
    is_cols = lambda x: x.startswith(("k_cols_solve", "k_cols_reg")) \
        and not x.startswith("k_cols_reg_batch")
    for i, s in enumerate(shorts):
        prev = shorts[i - 1] if i else ""
        nxt = shorts[i + 1] if i + 1 < len(shorts) else ""
        if s.startswith("k_AAt_tile"):
            # k_AAt_tile<HAS0, FUSE, BIG>: with the fused PCG direction when FUSE
            out.append("aat_fused" if _targs(s)[1:2] == ["true"] else "aat")
        elif s.startswith("k_rhs_tile") or s.startswith("k_rhs_batch"):
            out.append("rhs" if s.startswith("k_rhs_tile") else "rhs_batch")
        elif s.startswith("k_rhs"):
            # k_rhs<HASBAR, ...>: the right-hand side with HASBAR, else C y
            out.append("rhs" if _targs(s)[:1] == ["true"] else "apply_C")
        elif s.startswith(("k_tgemm64", "k_tgemm_lp<", "k_tgemm_lps<", "k_tgemm_stream")):
            args = _targs(s)
            mode = "f64" if s.startswith("k_tgemm64") else MODES.get(args[0], "f64")
            tx, ty = args[-2], args[-1]
            if tx == "double" and ty == "float":
                d = "fwd"
            elif tx == "float" and ty == "double":
                d = "inv"
            else:
                d = "inv" if (is_rows(prev) or is_cols(prev)) else "fwd"
            out.append(f"tgemm_{mode}_{d}")
        elif s.startswith("k_tgemm_rows_fwd"):
            # k_tgemm_rows_fwd<MODE, NTP, UPD>: the fused forward pass (with
            # the conjugate gradient update when UPD)
            args = _targs(s)
            pre = "update_" if args[2:3] == ["true"] else ""
            out.append(f"{pre}tgemm_rows_{MODES.get(args[0], 'f32')}_fwd")
        elif s.startswith("k_rows_tgemm_inv"):
            # k_rows_tgemm_inv<MODE, NTP>: the fused inverse pass
            out.append(f"rows_tgemm_{MODES.get(_targs(s)[0], 'f32')}_inv")
        elif s.startswith(("k_rows_batch", "k_rows_reg_batch", "k_cols_batch", "k_cols_reg_batch",
                           "k_AAt_batch", "k_tgemm_lp_batch")):
            out.append(s[2:].split("<")[0])
        elif is_rows(s):
            sfx = _prec_sfx(s)
            if is_cols(nxt):
                out.append("rows_fwd" + sfx)
            elif is_cols(prev):
                out.append("rows_inv" + sfx)
            else:
                out.append("rows_solve" + sfx)
        elif is_cols(s):
            out.append("cols_solve" + _prec_sfx(s))
        elif s.startswith("k_"):
            out.append(s[2:].split("<")[0])
        else:
            out.append(s[:60])
    return out


def _dispatches(db, counter=None):
    con = sqlite3.connect(db)
    if counter is None:
        rows = con.execute("select name, start, end from kernels order by start").fetchall()
        return [(n, (e - s) / 1e3) for n, s, e in rows]
    # a counter without a reduction in its expression has one row per shader
    # engine: sum the rows of each dispatch
    rows = con.execute("select name, sum(counter_value), min(start) from pmc_events "
                       "where counter_name=? group by pid, dispatch_id order by min(start)",
                       (counter,)).fetchall()
    return [(n, v) for n, v, _ in rows]


def kernel_stats(db):
    d = _dispatches(db)
    names = classify([n for n, _ in d])
    acc = collections.OrderedDict()
    for name, (_, us) in zip(names, d):
        a = acc.setdefault(name, [0, 0.0])
        a[0] += 1
        a[1] += us
    return {k: {"calls": c, "avg_us": t / c, "total_ms": t / 1e3} for k, (c, t) in acc.items()}


def counter_per_launch(db, counter):
    d = _dispatches(db, counter)
    names = classify([n for n, _ in d])
    acc = collections.defaultdict(list)
    for name, (_, v) in zip(names, d):
        acc[name].append(v)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def copy_kib(db, counter):
    """Largest reading of `counter` (KiB) over the calibration copy dispatches."""
    d = _dispatches(db, counter)
    vals = [v for n, v in d if "copyBuffer" in n or "copy" in n.lower()]
    return max(vals)


def cmd_stats(args):
    st = kernel_stats(args.db)
    tot = sum(v["total_ms"] for v in st.values())
    lines = [f"# Kernel trace: {args.title}", "", "Command:", "", "```", args.cmd, "```", "",
             "| kernel | calls | avg us | total ms | share |", "|---|---:|---:|---:|---:|"]
    for k, v in sorted(st.items(), key=lambda kv: -kv[1]["total_ms"]):
        lines.append(f"| {k} | {v['calls']} | {v['avg_us']:.1f} | {v['total_ms']:.2f} | "
                     f"{100 * v['total_ms'] / tot:.1f}% |")
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)


def cmd_traffic(args):
    # the copy moves 512 MiB each way (bench.py --calibrate-copy)
    true_kib = 512 * 1024
    kf = true_kib / copy_kib(args.cal_fetch, "FETCH_SIZE")
    kw = true_kib / copy_kib(args.cal_write, "WRITE_SIZE")
    fr = counter_per_launch(args.fetch, "FETCH_SIZE")
    wr = counter_per_launch(args.write, "WRITE_SIZE")
    kernels = {}
    for k in sorted(set(fr) | set(wr)):
        r = kf * fr.get(k, 0.0) * 1024
        w = kw * wr.get(k, 0.0) * 1024
        kernels[k] = {"read_bytes": r, "write_bytes": w, "bytes_per_launch": r + w}
    data = {}
    if args.merge and os.path.exists(args.out):
        with open(args.out) as f:
            data = json.load(f)
    from bench import kernel_sources_hash  # noqa: E402  (same hash as bench.py)
    h = kernel_sources_hash()
    if data.get("sources_hash") != h:
        data = {"sources_hash": h, "variants": {}}
    data["scale"] = {"fetch": kf, "write": kw}
    data["variants"][args.variant] = kernels
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps(kernels, indent=1))


def cmd_counters(args):
    # per dispatch, all counters side by side (every counter of a pass sees the
    # same dispatches in the same order)
    cols = {c: _dispatches(args.db, c) for c in args.counters}
    first = cols[args.counters[0]]
    names = classify([n for n, _ in first])
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for i, name in enumerate(names):
        vals = {c: cols[c][i][1] for c in args.counters}
        # launches that found the solve finished return at once: with --active C
        # they are left out of the averages (C = 0)
        if args.active and vals[args.active] == 0:
            continue
        for c, v in vals.items():
            acc[name][c].append(v)
    kernels = {k: dict({c: sum(v) / len(v) for c, v in d.items()},
                       launches=len(next(iter(d.values()))))
               for k, d in acc.items()}
    data = {}
    if args.merge and os.path.exists(args.out):
        with open(args.out) as f:
            data = json.load(f)
    data.setdefault("variants", {})[args.variant] = kernels
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    if args.md:
        cnames = sorted({c for v in data["variants"].values() for k in v.values() for c in k
                         if c != "launches"})
        lines = [f"# Counters: {args.title}", "", "Command (one pass per variant):", "", "```",
                 args.cmd, "```", "",
                 "Averages per launch over the launches counted (`launches`); rows of one "
                 "dispatch (one per shader engine) are summed.", "",
                 "| variant | kernel | launches | " + " | ".join(cnames) + " |",
                 "|---|---|---:|" + "---:|" * len(cnames)]
        for var, ks in data["variants"].items():
            for k, v in sorted(ks.items()):
                lines.append(f"| {var} | {k} | {v['launches']} | " +
                             " | ".join(f"{v.get(c, float('nan')):.6g}" for c in cnames) + " |")
        with open(args.md, "w") as f:
            f.write("\n".join(lines) + "\n")
    print(json.dumps(kernels, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    a = sub.add_parser("stats")
    a.add_argument("db")
    a.add_argument("--cmd", required=True)
    a.add_argument("--title", default="")
    a.add_argument("--out")
    b = sub.add_parser("traffic")
    b.add_argument("--variant", required=True)
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--cal-fetch", required=True)
    b.add_argument("--cal-write", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--merge", action="store_true")
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("--variant", required=True)
    c.add_argument("--counters", nargs="+", required=True)
    c.add_argument("--active", help="average only over dispatches where this counter is > 0")
    c.add_argument("--out", required=True)
    c.add_argument("--merge", action="store_true")
    c.add_argument("--md", help="also write a markdown table of every variant in --out")
    c.add_argument("--cmd", default="")
    c.add_argument("--title", default="")
    args = ap.parse_args(argv)
    if args.cmd_name == "stats":
        cmd_stats(args)
    elif args.cmd_name == "counters":
        cmd_counters(args)
    else:
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        sys.path.insert(0, root)
        cmd_traffic(args)


if __name__ == "__main__":
    main()
