"""Gate kernels one by one, and run-to-run determinism.

Every gate kind the library applies (RX, RY, RZ, CNOT, CZ, controlled
rotations, Pauli-string rotations) on every target qubit of a 10-qubit random
state, through qng_apply_circuit_dev, against the oracle's gate routine
(complex128: 1e-14 normwise; complex64: 2^-21, a few FP32 roundings of each
amplitude).  Determinism: the fused passes reduce every inner product in a
fixed order, so repeated steps are bitwise identical; the fused passes and the
one-kernel-per-primitive path agree to 1e-13 (complex128).
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

N = 10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2011_02991_amd as q
    c = q.Context(0)
    yield torch, q, c
    c.close()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300))


def gate_cases():
    rng = np.random.default_rng(91)
    cases = []
    for kind in (W.RX, W.RY, W.RZ):
        for q in range(N):
            cases.append(([kind, q, -1, 0], None))
    pairs = [(q, q + 1) for q in range(N - 1)] + [(q + 1, q) for q in range(N - 1)] + [(0, N - 1), (N - 1, 0), (2, 7)]
    for kind in (W.CNOT, W.CZ):
        for a, b in pairs:
            cases.append(([kind, a, b, -1], None))
    for kind in (W.CRX, W.CRY, W.CRZ):
        for a, b in pairs:
            cases.append(([kind, a, b, 0], None))
    for _ in range(12):
        letters = np.zeros(N, dtype=np.uint8)
        k = int(rng.integers(1, 5))
        letters[rng.choice(N, size=k, replace=False)] = rng.integers(1, 4, size=k)
        cases.append(([W.RPAULI, 0, -1, 0], letters[None, :]))
    return cases


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_every_gate_on_every_target(env, prec):
    torch, q, ctx = env
    psi0 = W.random_state(N, 92)
    dtype = torch.complex128 if prec == "c128" else torch.complex64
    tol = 1e-14 if prec == "c128" else 2.0 ** -21
    theta = np.array([1.234])
    worst = 0.0
    cases = gate_cases()
    for g, strings in cases:
        params = 1 if g[3] >= 0 else 0
        circ = q.Circuit(N, np.array([g], dtype=np.int32), params, strings=strings)
        st = torch.as_tensor(psi0, dtype=dtype).cuda().contiguous()
        ctx.apply_circuit_dev(circ, theta[:params], st.data_ptr(), prec=prec)
        torch.cuda.synchronize()
        want = oracle.apply_gate(N, g, theta, psi0, strings=strings)
        e = rel_err(st.cpu().numpy().astype(np.complex128), want)
        worst = max(worst, e)
        assert e <= tol, (g, None if strings is None else strings.tolist(), e)
    say(f"{prec}: {len(cases)} gates, worst {worst:.2e} (bound {tol:.1e})")


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_repeat_runs_are_bitwise_identical(env, prec):
    torch, q, ctx = env
    pr = W.scaled(W.config3, 16, 2, n_terms=12)
    pr.in_state = W.random_state(16, 93)
    circ = q.Circuit.from_problem(pr)
    runs = [ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state, prec=prec) for _ in range(3)]
    assert ctx.stats()["sweep_launches"] > 0
    for r in runs[1:]:
        for key in ("G", "grad", "dtheta"):
            assert np.array_equal(r[key], runs[0][key]), key
        assert r["E"] == runs[0]["E"]
    G1, T1 = ctx.metric(circ, pr.theta, in_state=pr.in_state, prec=prec)
    G2, T2 = ctx.metric(circ, pr.theta, in_state=pr.in_state, prec=prec)
    assert np.array_equal(G1, G2) and np.array_equal(T1, T2)
    if prec == "c128":
        ctx.set_option(q.OPT_FUSION, 0)
        try:
            ref = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
        finally:
            ctx.set_option(q.OPT_FUSION, 1)
        for key in ("G", "grad"):
            e = rel_err(runs[0][key], ref[key])
            say(f"fused vs per primitive {key}: {e:.2e}")
            assert e <= 1e-13, key
