"""Profiling helper for the fused sweep-pass kernels (k_sweep_reg and its builds).

Two modes:

  python profile_sweep.py run [--config 3] [--prec c64]
      One natural-gradient step of a workload without the G output (the passes
      bench.py times), preceded by one clone of a 512 MiB state with the
      library's own copy kernel (the calibration kernel for FETCH_SIZE /
      WRITE_SIZE).  Meant to run under rocprofv3 --pmc, one counter group per
      run.

  python profile_sweep.py summarize --kind {stats,traffic,counters} --out FILE DB...
      Summarise rocprofv3 databases into short text under profiles/:
      * stats:    per-kernel call counts and durations (kernel trace);
      * traffic:  FETCH_SIZE and WRITE_SIZE of the sweep kernel per launch,
                  scaled by what the same counters read for the 512 MiB copy,
                  tagged with the SHA-256 of the kernel source;
      * counters: any other counters of the sweep kernel, per wave.
"""
from __future__ import annotations

import argparse
import collections
import glob
import hashlib
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
KERNEL_SRC = os.path.join(ROOT, "paper_2011_02991_amd", "csrc", "sweep_kernels.hip")
COPY_BYTES = 512 * 2 ** 20


def run(args):
    import torch
    import paper_2011_02991_amd as qng
    import workloads as W
    ctx = qng.Context(0)
    src = torch.zeros(COPY_BYTES // 8, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    n_copy = (COPY_BYTES // 8).bit_length() - 1
    ctx.clone_state_dev(n_copy, src.data_ptr(), dst.data_ptr(), prec="c64")
    ctx.synchronize()
    del dst, src
    pr = W.CONFIGS[args.config]() if args.layers <= 0 else W.scaled(W.CONFIGS[args.config], 26, args.layers)
    print(f"profiling a step of {pr.name} ({args.prec}, exact products {args.exact_products})", flush=True)
    ctx.set_option(qng.OPT_TILE_QUBITS, args.tile)
    ctx.set_option(qng.OPT_F64_REGISTERS, args.f64_regs)
    ctx.set_option(qng.OPT_EXACT_PRODUCTS, args.exact_products)
    ctx.step(qng.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov, prec=args.prec, want_G=False)
    torch.cuda.synchronize()
    print(json.dumps({"workload": pr.name, "prec": args.prec, **ctx.stats()}), flush=True)
    ctx.close()


def _short(name: str) -> str:
    import re
    m = re.search(r"(k_\w+(?:<[^>]*>)?)", name)
    return m.group(1) if m else name[:60]


def _family(name: str) -> str:
    """The kernel's name without template arguments (each build of the sweep
    kernel has its own name: k_sweep_reg_real_exact, k_sweep_reg_states, ...)."""
    import re
    m = re.search(r"(k_\w+)", name)
    return m.group(1) if m else name[:60]


def _pmc(dbs):
    """Counter sums per kernel family, plus the calibration copy on its own.

    The calibration copy is the first dispatch of the library's copy kernel
    in each profiled process (the 512 MiB state clone that run() issues before
    the step; torch's fill of its source comes before it).  Only that one
    dispatch calibrates: the step itself launches copies of the same size
    (a state clone is a 512 MiB copy at n=26), which must not be summed in.
    """
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for db in dbs:
        con = sqlite3.connect(db)
        rows = list(con.execute("select name, counter_name, counter_value, dispatch_id from pmc_events"))
        if not rows:
            continue
        copies = [d for name, _, _, d in rows if _family(name) == "k_copy"]
        first = min(copies) if copies else None
        for name, cn, v, d in rows:
            f = "calib" if d == first else _family(name)
            agg[f][cn] += v
            disp[f].add(d)
    return agg, {k: len(v) for k, v in disp.items()}


def summarize(args):
    dbs = []
    for d in args.dbs:
        dbs += glob.glob(os.path.join(d, "**", "*.db"), recursive=True) if os.path.isdir(d) else [d]
    cmd = args.command or ""
    if args.kind == "stats":
        rows = collections.defaultdict(lambda: [0, 0.0])
        for db in dbs:
            con = sqlite3.connect(db)
            for name, dur in con.execute("select name, duration from kernels"):
                r = rows[_short(name)]
                r[0] += 1
                r[1] += dur
        total = sum(r[1] for r in rows.values()) or 1.0
        lines = [f"# Kernel trace summary: {args.title}", "", f"Command: `{cmd}`", "",
                 "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
        for name, (c, d) in sorted(rows.items(), key=lambda kv: -kv[1][1])[:15]:
            lines.append(f"| `{name[:80]}` | {c} | {d / 1e6:.1f} | {d / c / 1e3:.1f} | {100 * d / total:.1f} |")
        open(args.out, "w").write("\n".join(lines) + "\n")
    elif args.kind == "traffic":
        agg, nd = _pmc(dbs)
        sw, cp = agg[args.kernel], agg["calib"]
        f_fetch = COPY_BYTES / (cp["FETCH_SIZE"] * 1024) if cp.get("FETCH_SIZE") else None
        f_write = COPY_BYTES / (cp["WRITE_SIZE"] * 1024) if cp.get("WRITE_SIZE") else None
        n = nd.get(args.kernel, 1)
        fetch = sw.get("FETCH_SIZE", 0) * 1024 * (f_fetch or 1) / n
        write = sw.get("WRITE_SIZE", 0) * 1024 * (f_write or 1) / n
        out = {"kernel": args.kernel, "title": args.title, "command": cmd, "launches": n,
               "raw_fetch_kib": sw.get("FETCH_SIZE", 0), "raw_write_kib": sw.get("WRITE_SIZE", 0),
               "calib_fetch_kib": cp.get("FETCH_SIZE"), "calib_write_kib": cp.get("WRITE_SIZE"),
               "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
               "bytes_per_launch": fetch + write, "copy_scale_fetch": f_fetch, "copy_scale_write": f_write,
               "kernel_sha256": hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()}
        json.dump(out, open(args.out, "w"), indent=1)
    else:
        agg, nd = _pmc(dbs)
        sw = agg[args.kernel]
        waves = sw.get("SQ_WAVES", 0) or 1
        lines = [f"# Sweep-kernel counters: {args.title}", "", f"Command: `{cmd}`", "",
                 f"Kernel `{args.kernel}`, launches: {nd.get(args.kernel, 0)}; values per wave "
                 f"(SQ_WAVES = {waves:.0f})", "",
                 "| counter | per wave |", "|---|---|"]
        for k, v in sorted(sw.items()):
            lines.append(f"| {k} | {v / waves:.1f} |")
        with open(args.out, "a") as f:
            f.write("\n".join(lines) + "\n\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    r = sub.add_parser("run")
    r.add_argument("--config", type=int, default=3)
    r.add_argument("--prec", default="c64")
    r.add_argument("--tile", type=int, default=0)
    r.add_argument("--f64-regs", type=int, default=0)
    r.add_argument("--exact-products", type=int, default=1)
    r.add_argument("--layers", type=int, default=0, help="layers of a 26-qubit instance (0 = the full workload)")
    s = sub.add_parser("summarize")
    s.add_argument("--kind", choices=["stats", "traffic", "counters"], required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--command", default="")
    s.add_argument("--kernel", default="k_sweep_reg_real_exact",
                   help="traffic / counters: the kernel (name without template arguments)")
    s.add_argument("dbs", nargs="+")
    a = ap.parse_args()
    run(a) if a.mode == "run" else summarize(a)


if __name__ == "__main__":
    main()
