"""Benchmark: one natural-gradient step (G, grad E, dtheta) per timed step.

Default workload: 26 qubits, 8 layers of [RY on every qubit, RZ on every qubit,
CNOT chain], P = 416 parameters, 100-term random Pauli Hamiltonian, input
|0...0>, dt = 0.1, Tikhonov shift 1e-4.  The timed precision is complex64
state storage with FP64 inner products and FP64 solve ("chosen"); the same
step in complex128 ("plain FP64") is timed beside it.

Prints ONE JSON line (rank 0, N = 1 only; this build runs on a single GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 5])
    ap.add_argument("--prec", default="c64", choices=["c64", "c128"])
    ap.add_argument("--no-plain", action="store_true", help="skip the complex128 comparison leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU-baseline leg")
    ap.add_argument("--fusion", type=int, default=1)
    ap.add_argument("--gate-qubits", type=int, default=26)
    ap.add_argument("--tile", type=int, default=0, help="tile qubits of the fused passes (0 = library default)")
    ap.add_argument("--f64-regs", type=int, default=0, help="complex64: compute sweep tiles in FP64 registers")
    return ap.parse_args()


def time_steps(ctx, circ, pr, prec, steps, warmup):
    import torch
    for _ in range(warmup):
        ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, prec=prec, want_G=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for _ in range(steps):
        res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, prec=prec, want_G=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, res, ctx.stats()


def gate_apply_bandwidth(qng, ctx, n, prec):
    """Isolated single-gate apply at n qubits on one state, timed with HIP events
    on the library's stream.  Bytes: a rotation reads and writes every amplitude
    (2V); a CNOT swaps the half of the amplitudes whose control is 1 (V); a CZ
    negates the quarter with both bits set (V/2)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    dtype = torch.complex64 if prec == "c64" else torch.complex128
    state = torch.zeros(2 ** n, dtype=dtype, device=dev)
    state[0] = 1
    amp = 8 if prec == "c64" else 16
    V = amp * 2 ** n
    moved = {0: 2 * V, 1: 2 * V, 2: 2 * V, 3: V, 4: V // 2}
    results = []
    s = torch.cuda.Stream()
    ctx.set_stream(s.cuda_stream)
    try:
        with torch.cuda.stream(s):
            for kind in (0, 1, 2, 3, 4):
                for q in range(n if kind < 3 else n - 1):
                    g = [[kind, q, -1, 0]] if kind < 3 else [[kind, q, q + 1, -1]]
                    circ = qng.Circuit(n, np.array(g, dtype=np.int32))
                    th = [0.3] if kind < 3 else []
                    ctx.apply_circuit_dev(circ, th, state.data_ptr(), prec=prec)   # warm
                    reps = 5
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(s)
                    for _ in range(reps):
                        ctx.apply_circuit_dev(circ, th, state.data_ptr(), prec=prec)
                    e1.record(s)
                    s.synchronize()
                    ms = e0.elapsed_time(e1) / reps
                    results.append((kind, q, moved[kind] / (ms * 1e-3) / 1e9))
    finally:
        torch.cuda.synchronize()
        ctx.set_stream(None)
    rot = sorted(r[2] for r in results if r[0] < 3)
    fixed = sorted(r[2] for r in results if r[0] >= 3)
    return {"rotation_median_GBps": rot[len(rot) // 2], "rotation_worst_GBps": rot[0],
            "rotation_best_GBps": rot[-1], "fixed_median_GBps": fixed[len(fixed) // 2] if fixed else None,
            "n": n, "gates_measured": len(results), "frac_of_8TBps": rot[len(rot) // 2] / HBM_PEAK_GBS}


def cpu_baseline(pr):
    """The oracle, as it stands, on a bounded sample of the workload: one
    derivative state built gate by gate (the dominant cost of the oracle's
    step), extrapolated to the full step by its primitive counts."""
    import numpy as np
    import oracle
    cores = len(os.sched_getaffinity(0))
    n, M, P = pr.n_qubits, pr.n_gates, pr.n_params
    rot_pos = [k for k in range(M) if pr.gates[k, 3] >= 0]
    # sample: the derivative state of the parameter whose gate is at position
    # M - K (K gates after it), timed end to end
    K = 24
    sel_pos = rot_pos[-1]
    for k in reversed(rot_pos):
        if M - k >= K:
            sel_pos = k
            break
    p = int(pr.gates[sel_pos, 3])
    dim = 2 ** n
    t0 = time.perf_counter()
    psi = np.empty(dim, dtype=np.complex128)
    # the oracle's forward pass over the first gates: time per gate apply
    sub = type(pr)(**{**pr.__dict__, "gates": pr.gates[:K]})
    oracle.forward(sub)                      # first touch of the oracle's buffers
    t_fwd0 = time.perf_counter()
    a = oracle.forward(sub)
    t_apply = (time.perf_counter() - t_fwd0) / K
    t_ip0 = time.perf_counter()
    for _ in range(3):
        oracle.inner(a, a)
    t_inner = (time.perf_counter() - t_ip0) / 3
    elapsed = time.perf_counter() - t0
    # full oracle step = P derivative states (sum over p of the gates after it,
    # plus its prefix walked once) + P^2 inner products + H psi + solve
    applies = M + sum(M - k for k in rot_pos)
    inner = P * P + P
    est = applies * t_apply + inner * t_inner
    del psi, a, p
    return {"value": est, "unit": "s/step", "cores": cores, "kind": "oracle",
            "sample": f"{K} gate applies and 3 inner products of the oracle at n={n} (complex128, "
                      f"{elapsed:.1f} s), extrapolated to its {applies} applies and {inner} inner products per step"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2011_02991_amd as qng
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pr = W.CONFIGS[args.config]()
    log(f"workload {pr.name}: n={pr.n_qubits} P={pr.n_params} gates={pr.n_gates} terms={pr.n_terms}")
    circ = qng.Circuit.from_problem(pr)
    ctx = qng.Context(0)
    ctx.set_option(qng.OPT_FUSION, args.fusion)
    ctx.set_option(qng.OPT_TILE_QUBITS, args.tile)
    ctx.set_option(qng.OPT_F64_REGISTERS, args.f64_regs)
    ctx.set_option(qng.OPT_PROFILE, 0)
    t_chosen, res, st = time_steps(ctx, circ, pr, args.prec, args.steps, args.warmup)
    log(f"{args.prec}: {t_chosen:.3f} s/step  stats={st}")
    # hot-kernel timing: one more step with HIP events around every sweep launch
    ctx.set_option(qng.OPT_PROFILE, 1)
    ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, prec=args.prec, want_G=False)
    torch.cuda.synchronize()
    prof = ctx.stats()
    ctx.set_option(qng.OPT_PROFILE, 0)
    plain = None
    if not args.no_plain:
        other = "c128" if args.prec == "c64" else "c64"
        t_plain, _, st2 = time_steps(ctx, circ, pr, other, max(1, args.steps - 1), 1)
        plain = {"prec": other, "s_per_step": t_plain}
        log(f"{other}: {t_plain:.3f} s/step")
    gate = None
    if args.gate_qubits > 0:
        gate = gate_apply_bandwidth(qng, ctx, min(args.gate_qubits, pr.n_qubits), args.prec)
        log(f"gate apply: {gate}")
    cpu = None if args.no_cpu else cpu_baseline(pr)
    if prof["sweep_launches"] > 0 and prof["sweep_ms"] > 0:
        avg_ms = prof["sweep_ms"] / prof["sweep_launches"]
        per_launch_bytes = prof["sweep_bytes"] / prof["sweep_launches"]
        achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "sweep_pass",
                "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": per_launch_bytes}
    else:
        roof = None
    line = {
        "metric": "QNG step time (s) + gate-apply HBM GB/s at n=26,P=400; chosen vs plain FP64",
        "value": t_chosen, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_chosen * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 storage, f64 accumulate" if args.prec == "c64" else "c128",
        "data": "synthetic",
        "config": {"workload": pr.name, "n_qubits": pr.n_qubits, "P": pr.n_params, "gates": pr.n_gates,
                   "hamiltonian_terms": pr.n_terms, "precision": args.prec, "fusion": args.fusion,
                   "tile_qubits": args.tile or None, "f64_registers": bool(args.f64_regs)},
        "plain_fp64": plain, "gate_apply": gate, "roofline": roof, "cpu_baseline": cpu,
        "breakdown_ms": {"metric": st["metric_ms"], "grad": st["grad_ms"], "solve": st["solve_ms"]},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
