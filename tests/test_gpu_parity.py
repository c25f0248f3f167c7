"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerance for complex128 results is normwise relative: max|X_gpu - X_oracle| <=
1e-10 * max|X_oracle| for X in {G, T, grad E}, |E_gpu - E_oracle| <= 1e-10 *
max(1, |E|).  For dtheta the gate is the same bound relative to |dtheta| or, when
the shifted metric is ill conditioned, kappa(Re G + eps I) * 1e-14.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10
DEFAULT_FUSION = 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def qng():
    import torch  # noqa: F401  (loads the HIP runtime torch ships with, first)
    import paper_2011_02991_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(qng):
    c = qng.Context(0)
    yield c
    c.close()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(np.abs(b).max(initial=0.0), 1e-300)
    return float(np.abs(a - b).max(initial=0.0) / scale)


def check_step(res, want, pr, tol=TOL, label=""):
    eG = rel_err(res["G"], want["G"])
    eg = rel_err(res["grad"], want["grad"])
    eE = abs(res["E"] - want["E"]) / max(1.0, abs(want["E"]))
    g = want["G"].real + pr.tikhonov * np.eye(pr.n_params)
    kappa = np.linalg.cond(g) if pr.n_params else 1.0
    ed = rel_err(res["dtheta"], want["dtheta"])
    say(f"{label}: |dG|={eG:.2e} |dgrad|={eg:.2e} |dE|={eE:.2e} |ddtheta|={ed:.2e} kappa={kappa:.1e}")
    assert eG <= tol, eG
    assert eg <= tol, eg
    assert eE <= tol, eE
    assert ed <= max(tol, kappa * 1e-14) if tol == TOL else ed <= tol, ed


def run_step(ctx, qng, pr, prec="c128"):
    circ = qng.Circuit.from_problem(pr)
    return ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state, prec=prec)


@pytest.mark.parametrize("fusion", [0, 1])
def test_config1_full_step(ctx, qng, fusion):
    pr = W.config1()
    say(f"case: config1 step fusion={fusion}")
    ctx.set_option(qng.OPT_FUSION, fusion)
    try:
        res = run_step(ctx, qng, pr)
    finally:
        ctx.set_option(qng.OPT_FUSION, DEFAULT_FUSION)
    want = oracle.step(pr)
    check_step(res, want, pr, label=f"cfg1 fusion={fusion}")
    # metric entry point: G and T
    G, T = ctx.metric(qng.Circuit.from_problem(pr), pr.theta)
    assert rel_err(G, want["G"]) <= TOL
    assert rel_err(T, want["T"]) <= TOL


@pytest.mark.parametrize("n,ngates,seed", [(1, 6, 1), (2, 10, 2), (3, 24, 3), (5, 40, 4), (7, 60, 5), (9, 70, 6),
                                           (12, 50, 7), (14, 40, 8)])
def test_random_circuits(ctx, qng, n, ngates, seed):
    pr = W.random_circuit(n, ngates, seed, n_terms=7)
    if seed % 2 == 0:
        pr.in_state = W.random_state(n, seed)
    if seed % 3 == 0:
        pr = W.permute_params(pr, seed)
    say(f"case: random n={n} gates={ngates} seed={seed}")
    res = run_step(ctx, qng, pr)
    check_step(res, oracle.step(pr), pr, label=pr.name)


@pytest.mark.parametrize("cfg,n,layers", [(W.config2, 8, 4), (W.config3, 9, 3), (W.config5, 7, 3), (W.config1, 13, 2),
                                          (W.config3, 15, 2), (W.config2, 16, 2)])
def test_scaled_workloads(ctx, qng, cfg, n, layers):
    pr = W.scaled(cfg, n, layers, n_terms=12)
    say(f"case: {pr.name}")
    res = run_step(ctx, qng, pr)
    check_step(res, oracle.step(pr), pr, label=pr.name)


def test_edge_no_parameters(ctx, qng):
    """Only fixed gates: G is empty, E is still evaluated."""
    g = np.array([[W.CNOT, 0, 1, -1], [W.CZ, 1, 2, -1]], dtype=np.int32)
    pr = W.Problem("fixed", 3, g, np.zeros(0), np.array([[3, 3, 1]], np.uint8), np.array([0.7]),
                   in_state=W.random_state(3, 1))
    circ = qng.Circuit.from_problem(pr)
    E, grad = ctx.energy_grad(circ, pr.theta, in_state=pr.in_state)
    assert grad.shape == (0,)
    assert abs(E - oracle.energy(pr)) < 1e-12
    res = run_step(ctx, qng, pr)
    assert res["dtheta"].shape == (0,)


def test_edge_single_parameter(ctx, qng):
    g = np.array([[W.RX, 0, -1, 0]], dtype=np.int32)
    pr = W.Problem("one", 1, g, np.array([0.3]), np.array([[3], [2]], np.uint8), np.array([0.5, -1.1]))
    res = run_step(ctx, qng, pr)
    check_step(res, oracle.step(pr), pr, label="single")


def test_c64_config1_bound(ctx, qng):
    """complex64 storage, FP64 accumulation: errors per result against the FP64 oracle."""
    pr = W.config1()
    res = run_step(ctx, qng, pr, prec="c64")
    want = oracle.step(pr)
    eG, eg = rel_err(res["G"], want["G"]), rel_err(res["grad"], want["grad"])
    eE = abs(res["E"] - want["E"]) / max(1.0, abs(want["E"]))
    say(f"c64 cfg1: |dG|={eG:.2e} |dgrad|={eg:.2e} |dE|={eE:.2e}")
    assert eG < 2e-5 and eg < 2e-5 and eE < 2e-5


def test_device_entry_points(ctx, qng):
    import torch
    pr = W.scaled(W.config5, 6, 2, n_terms=9)
    pr.in_state = W.random_state(6, 3)
    circ = qng.Circuit.from_problem(pr)
    dev = torch.device("cuda:0")
    ins = torch.from_numpy(pr.in_state).to(dev)
    P = pr.n_params
    G = torch.zeros((P, P), dtype=torch.complex128, device=dev)
    T = torch.zeros(P, dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    ctx.set_stream(stream)
    try:
        ctx.metric_dev(circ, pr.theta, G.data_ptr(), T.data_ptr(), in_state_dev_ptr=ins.data_ptr())
        E = torch.zeros(1, dtype=torch.float64, device=dev)
        psi = torch.zeros(2 ** 6, dtype=torch.complex128, device=dev)
        ctx.energy_dev(circ, pr.theta, E.data_ptr(), psi.data_ptr(), in_state_dev_ptr=ins.data_ptr())
        grad = torch.zeros(P, dtype=torch.float64, device=dev)
        ctx.energy_grad_from_state_dev(circ, pr.theta, psi.data_ptr(), grad.data_ptr())
        torch.cuda.synchronize()
    finally:
        ctx.set_stream(None)
    want = oracle.step(pr)
    assert rel_err(G.cpu().numpy(), want["G"]) <= TOL
    assert rel_err(T.cpu().numpy(), want["T"]) <= TOL
    assert abs(E.item() - want["E"]) <= TOL * max(1, abs(want["E"]))
    assert rel_err(grad.cpu().numpy(), want["grad"]) <= TOL
    assert rel_err(psi.cpu().numpy(), want["psi"]) <= TOL


def test_errors_before_device_work(ctx, qng):
    pr = W.scaled(W.config1, 4, 1)
    circ = qng.Circuit.from_problem(pr)
    bad = np.full(16, 0.3, dtype=np.complex128)
    with pytest.raises(qng.QNGError) as e:
        ctx.step(circ, pr.theta, 0.1, 1e-4, in_state=bad)
    assert e.value.name == "QNG_E_NOT_NORMALIZED"
    ctx.set_mem_limit(1024)
    try:
        with pytest.raises(qng.QNGError) as e:
            ctx.step(circ, pr.theta, 0.1, 1e-4)
        assert e.value.name == "QNG_E_OUT_OF_MEMORY"
    finally:
        ctx.set_mem_limit(0)
    # eps = 0 on a metric with a zero row (leading RZ on |0>) -> not SPD
    g = np.array([[W.RZ, 0, -1, 0], [W.RY, 1, -1, 1]], dtype=np.int32)
    pr2 = W.Problem("zrow", 2, g, np.array([0.4, 0.9]), np.array([[3, 3]], np.uint8), np.array([1.0]))
    with pytest.raises(qng.QNGError) as e:
        ctx.step(qng.Circuit.from_problem(pr2), pr2.theta, 0.1, 0.0)
    assert e.value.name == "QNG_E_NOT_SPD"


@pytest.mark.parametrize("n_terms", [0, 1, 96, 97, 250])
def test_hamiltonian_chunks(ctx, qng, n_terms):
    """H psi is formed in one pass per chunk of 96 terms (the first chunk
    overwrites, later ones add): term counts at and around the chunk size, and
    none at all (E = 0, zero gradient)."""
    pr = W.random_circuit(9, 40, 4400 + n_terms, n_terms=max(n_terms, 1))
    if n_terms == 0:
        pr = W.Problem(**{**pr.__dict__, "pauli": np.zeros((0, 9), np.uint8), "coeff": np.zeros(0)})
    pr.in_state = W.random_state(9, 4401)
    say(f"case: {n_terms} Hamiltonian terms")
    E, grad = ctx.energy_grad(qng.Circuit.from_problem(pr), pr.theta, in_state=pr.in_state)
    if n_terms == 0:
        assert E == 0.0 and not grad.any()
        return
    Eo, go = oracle.energy_grad(pr)
    assert abs(E - Eo) <= TOL * max(1.0, abs(Eo)), (E, Eo)
    assert rel_err(grad, go) <= TOL
    E64, g64 = ctx.energy_grad(qng.Circuit.from_problem(pr), pr.theta, in_state=pr.in_state, prec="c64")
    bound = 4 * (pr.n_gates + n_terms) * 2.0 ** -24
    # complex64: each gate and each term rounds once in FP32 (4 M' 2^-24, M' = gates + terms),
    # E relative to the coefficient sum that bounds |H|
    assert abs(E64 - Eo) <= bound * max(1.0, np.abs(pr.coeff).sum()) and rel_err(g64, go) <= bound
