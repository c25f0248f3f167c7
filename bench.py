"""Benchmark: one natural-gradient step (G, grad E, dtheta) per timed step.

Default workload: 26 qubits, 8 layers of [RY on every qubit, RZ on every qubit,
CNOT chain], P = 416 parameters, 100-term random Pauli Hamiltonian, input
|0...0>, dt = 0.1, Tikhonov shift 1e-4.  The timed precision is complex64
state storage with every inner-product term formed and accumulated in FP64
and an FP64 solve ("chosen"); the same step in complex128 ("plain FP64") is
timed beside it, and the complex64 step with FP32 per-thread product shares as
a labelled variant.

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
# VALU peak of MI355X for FP64 and for non-packed FP32 (both 16 FMA lanes per
# SIMD per clock): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
KERNEL_SRC = os.path.join(ROOT, "paper_2011_02991_amd", "csrc", "sweep_kernels.hip")
# the sweep kernel the timed (no G output) steps launch, by storage and product setting
def sweep_kernel_name(prec, f64_regs, exact_products):
    if prec == "c64" and not f64_regs and exact_products:
        return "k_sweep_reg_real_exact"
    return "k_sweep_reg_real"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_pass_cfg3_traffic.json")


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
    ap.add_argument("--exact-products", type=int, default=1,
                    help="complex64 with FP32 registers: 1 (default) every inner-product term formed in FP64, "
                         "0 each thread's share formed in FP32")
    ap.add_argument("--no-with-g", action="store_true",
                    help="skip timing the step that also returns the complex G")
    ap.add_argument("--no-shares", action="store_true",
                    help="skip the complex64 leg with FP32 per-thread product shares")
    ap.add_argument("--no-states", action="store_true",
                    help="skip the derivative-state variant (P + 2 states kept, Gram matrix on the matrix cores)")
    ap.add_argument("--variants", action="store_true",
                    help="also time the cheaper metric variants (block-diagonal per layer, L only) on the workload")
    ap.add_argument("--batch", action="store_true",
                    help="also time the batched step (64-ansatz workload, n 12..22, and 48 ansaetze of n 8..16) "
                         "against one step call per ansatz")
    ap.add_argument("--gateset", action="store_true",
                    help="also measure controlled and Pauli-string rotations (isolated gate bandwidth at n=26 and "
                         "the step at n=24 next to plain rotations)")
    ap.add_argument("--block", type=int, default=0,
                    help="metric columns sharing one lambda sweep (1, 2 or 4; 0 = library default)")
    return ap.parse_args()


def time_steps(ctx, circ, pr, prec, steps, warmup, profile=False, want_G=False, need_G=True):
    """Time `steps` full steps (dtheta, grad E and E out; the metric enters the
    solve as Re G, so without a G output the library keeps the real parts of
    its inner products); with profile, HIP events bracket every sweep-pass
    launch on the library's stream during the timed steps themselves.  Returns
    the time, the last step's results (with G: one further untimed step with
    the G output when need_G) and the counters of the timed steps."""
    import torch
    import paper_2011_02991_amd as qng
    ctx.set_option(qng.OPT_PROFILE, 0)
    for _ in range(warmup):
        ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, prec=prec, want_G=False)
    torch.cuda.synchronize()
    ctx.set_option(qng.OPT_PROFILE, 1 if profile else 0)
    acc = {}
    t0 = time.perf_counter()
    res = None
    for _ in range(steps):
        res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, prec=prec, want_G=want_G)
        for k, v in ctx.stats().items():
            # counters add up over the steps; settings are the last step's
            acc[k] = v if k in ("block_columns", "tile_qubits", "target_tiles", "state_chunks") else acc.get(k, 0) + v
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ctx.set_option(qng.OPT_PROFILE, 0)
    if not want_G and need_G:
        res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, prec=prec, want_G=True)
    return dt, res, acc


def gate_apply_bandwidth(qng, ctx, n, prec):
    """Isolated single-gate apply at n qubits on one state, timed with HIP events
    on the library's stream.  Bytes: a rotation reads and writes every amplitude
    (2V); a CNOT swaps the half of the amplitudes whose control is 1 (V); a CZ
    negates the quarter with both bits set (V/2).  The attainable-bandwidth
    reference is the library's own clone kernel (read V, write V) on the same
    stream."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    dtype = torch.complex64 if prec == "c64" else torch.complex128
    state = torch.zeros(2 ** n, dtype=dtype, device=dev)
    state[0] = 1
    other = torch.empty_like(state)
    amp = 8 if prec == "c64" else 16
    V = amp * 2 ** n
    moved = {0: 2 * V, 1: 2 * V, 2: 2 * V, 3: V, 4: V // 2}
    results = []
    s = torch.cuda.Stream()
    ctx.set_stream(s.cuda_stream)
    reps = 5

    def timed(fn):
        fn()   # warm
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        s.synchronize()
        return e0.elapsed_time(e1) / reps

    try:
        with torch.cuda.stream(s):
            for kind in (0, 1, 2, 3, 4):
                for q in range(n if kind < 3 else n - 1):
                    g = [[kind, q, -1, 0]] if kind < 3 else [[kind, q, q + 1, -1]]
                    circ = qng.Circuit(n, np.array(g, dtype=np.int32))
                    th = [0.3] if kind < 3 else []
                    ms = timed(lambda: ctx.apply_circuit_dev(circ, th, state.data_ptr(), prec=prec))
                    results.append((kind, q, moved[kind] / (ms * 1e-3) / 1e9))
            copy_ms = timed(lambda: ctx.clone_state_dev(n, state.data_ptr(), other.data_ptr(), prec=prec))
    finally:
        torch.cuda.synchronize()
        ctx.set_stream(None)
    copy_GBps = 2 * V / (copy_ms * 1e-3) / 1e9
    rot = sorted(r[2] for r in results if r[0] < 3)
    fixed = sorted(r[2] for r in results if r[0] >= 3)
    names = {0: "RX", 1: "RY", 2: "RZ", 3: "CNOT", 4: "CZ"}
    per_q = {names[k]: [round(r[2], 1) for r in results if r[0] == k] for k in names}
    return {"rotation_median_GBps": rot[len(rot) // 2], "rotation_worst_GBps": rot[0],
            "rotation_best_GBps": rot[-1], "fixed_median_GBps": fixed[len(fixed) // 2] if fixed else None,
            "n": n, "gates_measured": len(results), "frac_of_8TBps": rot[len(rot) // 2] / HBM_PEAK_GBS,
            "worst_frac_of_8TBps": rot[0] / HBM_PEAK_GBS,
            "copy_GBps": copy_GBps, "copy_kernel": "library clone (qng_clone_state_dev)",
            "rotation_median_frac_of_copy": rot[len(rot) // 2] / copy_GBps, "per_q_GBps": per_q}


def precision_report(pr, res, ref, prec, ref_prec):
    """Normwise differences of one precision's step against the other's (the
    complex128 path is the FP64 reference at this size; it is pinned to the
    oracle on sampled parameters by the full-size parity tests)."""
    import numpy as np

    def rel(a, b):
        return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))

    g = ref["G"].real + pr.tikhonov * np.eye(pr.n_params)
    return {"prec": prec, "reference": ref_prec, "max_abs_dG": float(np.abs(res["G"] - ref["G"]).max()),
            "rel_dG": rel(res["G"], ref["G"]), "max_abs_dgrad": float(np.abs(res["grad"] - ref["grad"]).max()),
            "rel_dgrad": rel(res["grad"], ref["grad"]), "abs_dE": abs(res["E"] - ref["E"]),
            "max_abs_ddtheta": float(np.abs(res["dtheta"] - ref["dtheta"]).max()),
            "rel_ddtheta": rel(res["dtheta"], ref["dtheta"]), "kappa_shifted_metric": float(np.linalg.cond(g))}


def sample_params(P: int, seed: int):
    """First, last and one run of two consecutive parameter indices."""
    import numpy as np
    rng = np.random.default_rng(seed)
    a = int(rng.integers(1, P - 2))
    return sorted({0, P - 1, a, a + 1})


def cpu_baseline(pr, gpu_results):
    """The oracle, as it stands, on a bounded sample of the workload, by its own
    route: derivative states of a few sampled parameters (rolling prefix, then
    each state's suffix, gate by gate), their Gram matrix, T, H psi and the
    gradient entries (numpy library products), timed on the host's cores.
    The full step is extrapolated from the measured rates: gate applies by the
    oracle's own count (the prefix walk plus every derivative state's suffix),
    the P x P Gram matrix at the rate its library product reaches on a
    32-state block, the gradient products linearly in P.  The sampled entries
    also pin the GPU results (gpu_results: precision -> step results) to the
    oracle."""
    import numpy as np
    import oracle
    cores = len(os.sched_getaffinity(0))
    n, M, P = pr.n_qubits, pr.n_gates, pr.n_params
    pos_of = {int(pr.gates[k, 3]): k for k in range(M) if pr.gates[k, 3] >= 0}
    sel = sample_params(P, 7001)
    t0 = time.perf_counter()
    D, psi = oracle.derivative_states(pr, sel)
    t_states = time.perf_counter() - t0
    t1 = time.perf_counter()
    G, T, _ = oracle.metric_from_states(D, psi)
    t_gram_sample = time.perf_counter() - t1
    t1 = time.perf_counter()
    hpsi = oracle.apply_hamiltonian(pr, psi)
    t_h = time.perf_counter() - t1
    t1 = time.perf_counter()
    E = float(np.vdot(psi, hpsi).real)
    grad = 2.0 * (D @ hpsi.conj()).real
    t_gradprod = (time.perf_counter() - t1) / len(sel)
    del D, psi, hpsi
    # Gram-matrix rate of the oracle's library product on a 32-state block
    rng = np.random.default_rng(7002)
    blk = rng.standard_normal((32, 2 ** min(n, 21))) + 1j * rng.standard_normal((32, 2 ** min(n, 21)))
    blk_psi = blk[0].copy()
    t1 = time.perf_counter()
    oracle.metric_from_states(blk, blk_psi)
    t_blk = time.perf_counter() - t1
    gram_rate = 8.0 * 32 * 32 * blk.shape[1] / t_blk          # real flops per second
    del blk, blk_psi
    measured = time.perf_counter() - t0
    applies_sample = M + sum(M - pos_of[p] for p in sel)
    applies_full = M + sum(M - pos_of[p] for p in range(P))
    t_apply = t_states / applies_sample
    est = (applies_full * t_apply + 8.0 * P * P * (2 ** n) / gram_rate + t_h + P * t_gradprod)
    errors = {}
    ix = np.ix_(sel, sel)
    for prec, res in gpu_results.items():
        if res is None or res.get("G") is None:
            continue
        gs = res["G"][ix]
        errors[prec] = {
            "sampled_params": sel,
            "rel_dG": float(np.abs(gs - G).max() / np.abs(G).max()),
            "rel_dgrad": float(np.abs(res["grad"][sel] - grad).max() / np.abs(grad).max()),
            "abs_dE": abs(res["E"] - E)}
    base = {"value": est, "unit": "s/step", "cores": cores, "kind": "oracle",
            "sample": f"oracle derivative states of parameters {sel} at n={n} (complex128: {applies_sample} gate "
                      f"applies in {t_states:.1f} s, {t_apply * 1e3:.1f} ms each), their Gram matrix "
                      f"({t_gram_sample:.2f} s), H psi ({t_h:.1f} s) and gradient entries; {measured:.1f} s "
                      f"measured; extrapolated to the full step: {applies_full} gate applies, the {P}x{P} Gram "
                      f"matrix at {gram_rate / 1e9:.1f} GFLOP/s (library product on a 32-state block), {P} "
                      f"gradient products"}
    return base, errors


def full_oracle_small(W):
    """The whole oracle step (every derivative state, Gram matrix, gradient,
    solve) on the 10-qubit, 80-parameter workload, timed."""
    import oracle
    pr = W.config1()
    t0 = time.perf_counter()
    oracle.step(pr)
    return {"workload": pr.name, "s_per_step": time.perf_counter() - t0}


def metric_variants(qng, ctx, circ, pr, prec, reps=2):
    """Metric time (s) of the full G and of the cheaper variants on the same
    workload: block-diagonal with one block per layer (parameters of a layer in
    gate order) and the L-only matrix."""
    import numpy as np
    import torch
    layers = max(1, int(round(pr.n_params / (2 * pr.n_qubits))))
    blocks = np.repeat(np.arange(layers), -(-pr.n_params // layers))[:pr.n_params].astype(np.int32)

    def timed():
        ctx.metric(circ, pr.theta, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.metric(circ, pr.theta, prec=prec)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    out = {"full_s": timed()}
    ctx.set_metric_blocks(blocks)
    try:
        out["block_diagonal_s"] = timed()
        out["block_diagonal_elements"] = ctx.stats()["elements"]
    finally:
        ctx.set_metric_blocks(None)
    ctx.set_option(qng.OPT_METRIC_KIND, 1)
    try:
        out["l_only_s"] = timed()
    finally:
        ctx.set_option(qng.OPT_METRIC_KIND, 0)
    out["blocks"] = f"{layers} blocks of {pr.n_params // layers} parameters (one per layer)"
    log(f"metric variants: {out}")
    return out


def batched_steps(qng, ctx, prec, reps=2):
    """qng_step_batched (graph replay, no G outputs) against one qng_step per
    ansatz, wall time per step of all members after one warm-up call each way:
    the 64-ansatz workload (n 12..22, 2..8 layers of RY, RZ, CNOT chain, 30
    terms) and 48 ansaetze of n 8..16 (2..6 layers), where one ansatz alone
    cannot fill the GPU."""
    import numpy as np
    import torch
    import workloads as W
    rng = np.random.default_rng(7201)
    small = [W.make_problem(f"small{b}", int(rng.integers(8, 17)), int(rng.integers(2, 7)), (W.RY, W.RZ),
                            "cnot_chain", 12, 7300 + b) for b in range(48)]
    out = {}
    ctx.set_option(qng.OPT_GRAPH, 1)
    for name, probs in (("cfg4_64_ansaetze_n12_22", W.config4()), ("small_48_ansaetze_n8_16", small)):
        circs = [qng.Circuit.from_problem(p) for p in probs]
        ths = [p.theta for p in probs]
        dt, eps = probs[0].dt, probs[0].tikhonov

        def batched():
            ctx.step_batched(circs, ths, dt, eps, prec=prec, want_G=False)

        def singles():
            for c, t, p in zip(circs, ths, probs):
                ctx.step(c, t, p.dt, p.tikhonov, prec=prec, want_G=False)

        times = {}
        for key, fn in (("batched_s", batched), ("one_call_per_ansatz_s", singles)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            times[key] = (time.perf_counter() - t0) / reps
        out[name] = {"members": len(probs), "params": int(sum(p.n_params for p in probs)), "prec": prec, **times,
                     "speedup": times["one_call_per_ansatz_s"] / times["batched_s"]}
    return out


def extended_gates(qng, ctx, prec, n_gate=26, n_step=24, layers=2, reps=2):
    """Controlled (CRX/CRY/CRZ) and Pauli-string rotations.

    Isolated apply at n_gate qubits (HIP events on the library's stream):
    a controlled rotation reads and writes the half of the amplitudes whose
    control is 1 (V bytes); a string rotation reads and writes every amplitude
    (2V).  Then the step at n_step qubits for the controlled ring ansatz and the
    ZZ / X Y..Y X string ansatz (both on the fused passes: controlled rotations
    with their own handlers, strings rewritten into basis rotations, CNOTs and
    an RZ), next to a plain RY/RZ + CNOT ansatz with the same P on the
    per-primitive kernels and on the fused passes."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    dtype = torch.complex64 if prec == "c64" else torch.complex128
    n = n_gate
    state = torch.zeros(2 ** n, dtype=dtype, device=dev)
    state[0] = 1
    V = (8 if prec == "c64" else 16) * 2 ** n
    cases = []
    for kind in (W.CRX, W.CRY, W.CRZ):
        for q in (0, 5, 12, n - 2):
            cases.append((f"CR{'XYZ'[kind - W.CRX]}({q},{q + 1})", [[kind, q, q + 1, 0]], None, V))
            cases.append((f"CR{'XYZ'[kind - W.CRX]}({q + 1},{q})", [[kind, q + 1, q, 0]], None, V))
    for name, letters in (("ZZ(0,1)", {0: 3, 1: 3}), ("ZZ(12,13)", {12: 3, 13: 3}), ("XX(0,1)", {0: 1, 1: 1}),
                          ("XYYX(10..13)", {10: 1, 11: 2, 12: 2, 13: 1}), ("X..X (all)", {q: 1 for q in range(n)}),
                          ("Y(n-1)Z(0)", {n - 1: 2, 0: 3})):
        st_ = np.zeros((1, n), dtype=np.uint8)
        for q, l in letters.items():
            st_[0, q] = l
        cases.append((name, [[W.RPAULI, 0, -1, 0]], st_, 2 * V))
    iso = []
    s = torch.cuda.Stream()
    ctx.set_stream(s.cuda_stream)
    try:
        with torch.cuda.stream(s):
            for name, g, strings, moved in cases:
                circ = qng.Circuit(n, np.array(g, dtype=np.int32), 1, strings=strings)
                ctx.apply_circuit_dev(circ, [0.3], state.data_ptr(), prec=prec)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                for _ in range(5):
                    ctx.apply_circuit_dev(circ, [0.3], state.data_ptr(), prec=prec)
                e1.record(s)
                s.synchronize()
                ms = e0.elapsed_time(e1) / 5
                iso.append({"gate": name, "ms": ms, "GBps": moved / (ms * 1e-3) / 1e9})
    finally:
        torch.cuda.synchronize()
        ctx.set_stream(None)
    del state

    def step_time(pr, fusion):
        c = qng.Circuit.from_problem(pr)
        ctx.set_option(qng.OPT_FUSION, fusion)
        try:
            ctx.step(c, pr.theta, pr.dt, pr.tikhonov, prec=prec, want_G=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.step(c, pr.theta, pr.dt, pr.tikhonov, prec=prec, want_G=False)
            torch.cuda.synchronize()
            st = ctx.stats()
        finally:
            ctx.set_option(qng.OPT_FUSION, 1)
        return {"workload": pr.name, "P": pr.n_params, "fusion": fusion, "s_per_step": (time.perf_counter() - t0) / reps,
                "elements": st["elements"], "sweep_launches": st["sweep_launches"],
                "other_launches": st["other_launches"]}

    plain = W.make_problem(f"ry_rz_cnot_n{n_step}_L{layers}", n_step, layers, (W.RY, W.RZ), "cnot_chain", 30, 5401)
    steps = [step_time(W.controlled_layers(n_step, layers, 30, 5402), 1),
             step_time(W.string_layers(n_step, layers, 30, 5403), 1),
             step_time(plain, 0), step_time(plain, 1)]
    out = {"isolated_n": n, "isolated": iso, "steps_n": n_step, "steps": steps}
    log(f"extended gates: {out}")
    return out


def traffic_per_launch(kernel):
    """HBM bytes per sweep launch from the committed FETCH_SIZE/WRITE_SIZE counter
    summary, if it was taken on the current kernel source and for this kernel
    (else None)."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        h = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if t.get("kernel_sha256") != h or t.get("kernel") != kernel:
            return None
        return t["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


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
    ctx.set_option(qng.OPT_EXACT_PRODUCTS, args.exact_products)
    ctx.set_option(qng.OPT_BLOCK_COLUMNS, args.block)
    t_chosen, res, st = time_steps(ctx, circ, pr, args.prec, args.steps, args.warmup, profile=True,
                                   need_G=not args.no_plain or not args.no_cpu)
    log(f"{args.prec}: {t_chosen:.3f} s/step  stats={st}")
    plain = precision = res_other = None
    if not args.no_plain:
        other = "c128" if args.prec == "c64" else "c64"
        t_plain, res_other, st2 = time_steps(ctx, circ, pr, other, max(1, args.steps - 1), 1)
        plain = {"prec": other, "s_per_step": t_plain}
        log(f"{other}: {t_plain:.3f} s/step")
        if args.prec == "c64":
            precision = precision_report(pr, res, res_other, "c64", "c128")
        else:
            precision = precision_report(pr, res_other, res, "c64", "c128")
        log(f"precision: {precision}")
    # the same step asked for the complex G as well (full inner products)
    t_with_G = None
    if not args.no_with_g:
        t_with_G, _, _ = time_steps(ctx, circ, pr, args.prec, max(1, args.steps - 1), 0, want_G=True)
        log(f"{args.prec} with the G output: {t_with_G:.3f} s/step")
    shares = None
    if args.prec == "c64" and not args.f64_regs and args.exact_products and not args.no_shares:
        # the narrower arithmetic: each thread's share of a product formed in FP32
        ctx.set_option(qng.OPT_EXACT_PRODUCTS, 0)
        try:
            t_sh, res_sh, _ = time_steps(ctx, circ, pr, "c64", max(1, args.steps - 1), 1)
        finally:
            ctx.set_option(qng.OPT_EXACT_PRODUCTS, args.exact_products)
        shares = {"s_per_step": t_sh,
                  "precision_errors": precision_report(pr, res_sh, res_other, "c64", "c128") if plain else None,
                  "max_abs_dG_vs_exact_products": float(abs(res_sh["G"] - res["G"]).max())}
        log(f"c64 with FP32 thread shares: {shares}")
    states = None
    if not args.no_states:
        # the derivative-state variant of the metric: the same step with every
        # column's derivative state kept and all inner products as one Gram matrix
        ctx.set_option(qng.OPT_METHOD, 1)
        try:
            t_st, res_st, st_st = time_steps(ctx, circ, pr, args.prec, max(1, args.steps - 1), 1, profile=True)
            V = (8 if args.prec == "c64" else 16) * 2 ** pr.n_qubits
            nst = max(1, args.steps - 1)
            states = {"s_per_step": t_st, "kept_states_GiB": (pr.n_params + 2) * V / 2 ** 30,
                      "sweep_ms_per_step": st_st["sweep_ms"] / nst, "metric_ms_per_step": st_st["metric_ms"] / nst,
                      "rel_ddtheta_vs_recurrence": float(abs(res_st["dtheta"] - res["dtheta"]).max()
                                                         / abs(res["dtheta"]).max())}
            if res.get("G") is not None and res_st.get("G") is not None:
                states["max_abs_dG_vs_recurrence"] = float(abs(res_st["G"] - res["G"]).max())
            # the memory dial: a quarter of the columns per chunk (two chunks
            # kept at once), chunk i paired with every lower chunk
            chunk = -(-(pr.n_params - 1) // 4)
            ctx.set_option(qng.OPT_STATE_CHUNK, chunk)
            t_ch, res_ch, st_ch = time_steps(ctx, circ, pr, args.prec, 1, 1, need_G=False)
            states["chunked"] = {"chunk_columns": chunk, "chunks": st_ch["state_chunks"],
                                 "kept_states_GiB": (2 * chunk + 3) * V / 2 ** 30, "s_per_step": t_ch,
                                 "rel_ddtheta_vs_unchunked": float(abs(res_ch["dtheta"] - res_st["dtheta"]).max()
                                                                   / abs(res_st["dtheta"]).max())}
        except qng.QNGError as e:
            states = {"error": str(e)}
        finally:
            ctx.set_option(qng.OPT_STATE_CHUNK, 0)
            ctx.set_option(qng.OPT_METHOD, 0)
        log(f"derivative-state variant: {states}")
    gate = None
    if args.gate_qubits > 0:
        gate = gate_apply_bandwidth(qng, ctx, min(args.gate_qubits, pr.n_qubits), args.prec)
        log(f"gate apply: {gate}")
    variants = metric_variants(qng, ctx, circ, pr, args.prec) if args.variants else None
    gateset = extended_gates(qng, ctx, args.prec) if args.gateset else None
    batch = batched_steps(qng, ctx, "c128") if args.batch else None
    if batch:
        log(f"batched steps: {batch}")
    cpu = oracle_errors = small = None
    if not args.no_cpu:
        cpu, oracle_errors = cpu_baseline(pr, {args.prec: res, **({plain["prec"]: res_other} if plain else {})})
        small = full_oracle_small(W)
        cpu["full_oracle_small_workload"] = small
        log(f"cpu baseline: {cpu}")
        log(f"oracle-pinned errors on sampled parameters: {oracle_errors}")
    roof = None
    kname = sweep_kernel_name(args.prec, args.f64_regs, args.exact_products)
    if st.get("sweep_launches", 0) > 0 and st.get("sweep_ms", 0) > 0:
        nl = st["sweep_launches"]
        avg_ms = st["sweep_ms"] / nl
        flops = st["sweep_flops"] / nl
        bytes_ = st["sweep_bytes"] / nl
        achieved = flops / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / VALU_PEAK_TFLOPS, "traffic": traffic_per_launch(kname), "kernel": kname,
                "avg_launch_ms": avg_ms, "launches": nl, "algorithmic_flops_per_launch": flops,
                "algorithmic_bytes_per_launch": bytes_,
                "hbm_achieved_GBps": bytes_ / (avg_ms * 1e-3) / 1e9,
                "hbm_frac": bytes_ / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    line = {
        "metric": "QNG step time (s) + gate-apply HBM GB/s at n=26,P=400; chosen vs plain FP64",
        "value": t_chosen, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_chosen * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": ("c128" if args.prec == "c128" else
                  "c64 storage, f64 registers" if args.f64_regs else
                  "c64 storage, f64 products and accumulation" if args.exact_products else
                  "c64 storage, f32 per-thread product shares, f64 accumulation"),
        "data": "synthetic",
        "config": {"workload": pr.name, "n_qubits": pr.n_qubits, "P": pr.n_params, "gates": pr.n_gates,
                   "hamiltonian_terms": pr.n_terms, "precision": args.prec, "fusion": args.fusion,
                   "tile_qubits": args.tile or None, "f64_registers": bool(args.f64_regs),
                   "exact_products": bool(args.exact_products),
                   "block_columns": st.get("block_columns")},
        "plain_fp64": plain, "precision_errors": precision, "oracle_pinned_errors": oracle_errors,
        "c64_fp32_product_shares": shares, "derivative_state_variant": states,
        "step_with_G_output_s": t_with_G, "gate_apply": gate, "roofline": roof, "cpu_baseline": cpu,
        "metric_variants": variants, "extended_gates": gateset, "batched_steps": batch,
        "breakdown_ms": {k: st[k] / args.steps for k in ("metric_ms", "grad_ms", "solve_ms")},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
