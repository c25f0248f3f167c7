"""Parameters shared by several rotations, against the FP64 CPU oracle.

The oracle differentiates a shared angle through every gate that carries it
(the sum of the gates' derivative terms); the library computes the metric,
T and the gradient per rotation and contracts them (J^T G J, J^T T,
J^T grad).  complex128 results must match to 1e-10 normwise (Delta theta:
kappa(Re G + eps I) * 1e-14 when larger); complex64 to the bound
4 M 2^-24.  Workloads: layers of RX and RZ with one angle per layer and gate
type (n = 6 and 12, the latter through the fused two-column sweeps), random
circuits with parameters merged at random (input state, CZ and CNOT, RX/RY/RZ),
the energy gradient on the device (autograd), and a batch with shared and
unshared members.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def check(res, want, pr, tol, label):
    eG, eg = rel_err(res["G"], want["G"]), rel_err(res["grad"], want["grad"])
    eE = abs(res["E"] - want["E"]) / max(1.0, abs(want["E"]))
    ed = rel_err(res["dtheta"], want["dtheta"])
    kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(pr.n_params))
    say(f"{label}: P={pr.n_params} |dG|={eG:.2e} |dgrad|={eg:.2e} |dE|={eE:.2e} |ddtheta|={ed:.2e} kappa={kappa:.1e}")
    assert eG <= tol and eg <= tol and eE <= tol, (eG, eg, eE)
    assert ed <= max(tol, kappa * tol * 1e-4), ed


CASES = [
    ("layers n=6 L=3", lambda: W.layer_shared(6, 3, 8, 3101)),
    ("layers n=12 L=2", lambda: W.layer_shared(12, 2, 9, 3102)),
    ("random n=7 merged", lambda: W.share_params(W.random_circuit(7, 50, 3103, n_terms=6), 9, 3104)),
    ("random n=9 merged, input state", lambda: W.share_params(W.random_circuit(9, 44, 3105, n_terms=6), 5, 3106)),
]


@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_shared_step_complex128(env, label, make):
    torch, q, ctx = env
    pr = make()
    if "input state" in label:
        pr.in_state = W.random_state(pr.n_qubits, 3107)
    say(f"case: {label} (n={pr.n_qubits}, P={pr.n_params}, rotations={(pr.gates[:, 3] >= 0).sum()})")
    circ = q.Circuit.from_problem(pr)
    res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
    want = oracle.step(pr)
    check(res, want, pr, TOL, label)
    G, T = ctx.metric(circ, pr.theta, in_state=pr.in_state)
    Go, To = oracle.metric(pr)
    assert rel_err(G, Go) <= TOL and rel_err(T, To) <= TOL


def test_shared_complex64_bound(env):
    torch, q, ctx = env
    pr = W.layer_shared(12, 2, 9, 3102)
    res = ctx.step(q.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov, prec="c64")
    want = oracle.step(pr)
    bound = 4 * pr.n_gates * 2.0 ** -24
    eG, eg = rel_err(res["G"], want["G"]), rel_err(res["grad"], want["grad"])
    say(f"c64 shared: |dG|={eG:.2e} |dgrad|={eg:.2e} (bound {bound:.1e})")
    assert eG <= bound and eg <= bound


def test_shared_autograd_device_gradient(env):
    """energy as a torch.autograd.Function: the backward's gradient (contracted
    on the device) against the oracle."""
    torch, q, ctx = env
    from paper_2011_02991_amd import torch_energy as te
    pr = W.share_params(W.random_circuit(8, 48, 3108, n_terms=7), 7, 3109)
    th = torch.tensor(pr.theta, dtype=torch.float64, requires_grad=True)
    E = te.energy(ctx, q.Circuit.from_problem(pr), th)
    E.backward()
    Eo, go = oracle.energy_grad(pr)
    say(f"autograd shared: |dE|={abs(E.item() - Eo):.2e} |dgrad|={rel_err(th.grad.numpy(), go):.2e}")
    assert abs(E.item() - Eo) <= TOL * max(1.0, abs(Eo))
    assert rel_err(th.grad.numpy(), go) <= TOL


def test_shared_in_a_batch(env):
    torch, q, ctx = env
    probs = [W.layer_shared(6, 2, 6, 3110), W.scaled(W.config1, 7, 2, seed=3111),
             W.share_params(W.random_circuit(8, 40, 3112, n_terms=5), 6, 3113)]
    circs = [q.Circuit.from_problem(p) for p in probs]
    res = ctx.step_batched(circs, [p.theta for p in probs], probs[0].dt, probs[0].tikhonov)
    for b, (r, p) in enumerate(zip(res, probs)):
        check(r, oracle.step(p), p, TOL, f"batch member {b}")
