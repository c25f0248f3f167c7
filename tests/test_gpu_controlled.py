"""Controlled rotations CRX/CRY/CRZ against the FP64 CPU oracle.

A controlled rotation's column uses the generator |1><1|_c (x) sigma_t in
every product and seed, and its diagonal L_ii is 1/4 Prob(control = 1) of the
state before the gate (Sec. 2) rather than 1/4.  These circuits run on the
fused sweep passes (the kernels with the second handler word: the control's
value per register is a mask, the adjoint a plane rotation that is the
identity where the control is 0, the generator a masked lambda) and, with
fusion off, on the per-primitive kernels.  complex128 results must match the
oracle to 1e-10 normwise (Delta theta: kappa(Re G + eps I) * 1e-14 when
larger); complex64 to 4 M 2^-24 (M gates each rounding the state once in FP32
storage, FP64 sums); fused against per-primitive kernels on the same inputs
to 1e-12 (complex128).

Workloads: random circuits mixing CRX/CRY/CRZ with plain rotations, CNOT and
CZ (n = 2 .. 14, with and without an input state, permuted parameters), the
ring ansatz of RY layers and controlled rotations, shared angles, the
block-diagonal and L-only variants, the device entry points, the autograd
energy and, at n = 22, sampled metric entries and gradient entries; the
fused passes with one and two columns per sweep, FP64 and FP32 registers,
FP32 shares and exact FP64 products, real-part products, controls outside the
tile (registers of 13-16 qubits with tiles of 11 and 12).
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
    assert ed <= max(tol, kappa * 1e-14), ed


CASES = [(2, 12, 5201), (3, 24, 5202), (5, 40, 5203), (7, 60, 5204), (10, 70, 5205), (14, 50, 5206)]


@pytest.mark.parametrize("n,ngates,seed", CASES)
def test_random_controlled_circuits(env, n, ngates, seed):
    torch, q, ctx = env
    pr = W.controlled_circuit(n, ngates, seed, n_terms=7)
    if seed % 2 == 0:
        pr.in_state = W.random_state(n, seed)
    if seed % 3 == 0:
        pr = W.permute_params(pr, seed)
    ncr = int((pr.gates[:, 0] >= W.CRX).sum())
    say(f"case: {pr.name} ({ncr} controlled rotations)")
    assert ncr > 0
    circ = q.Circuit.from_problem(pr)
    res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
    st = ctx.stats()
    assert st["sweep_launches"] > 0 or pr.n_params < 2
    want = oracle.step(pr)
    check(res, want, pr, TOL, pr.name)
    G, T = ctx.metric(circ, pr.theta, in_state=pr.in_state)
    assert rel_err(G, want["G"]) <= TOL and rel_err(T, want["T"]) <= TOL


def test_diagonal_is_quarter_control_probability(env):
    """L_ii = 1/4 Prob(control = 1) (Sec. 2): the L-only metric's diagonal
    against the probabilities of the oracle's states before each gate."""
    torch, q, ctx = env
    pr = W.controlled_layers(6, 2, 5, 5207)
    pr.in_state = W.random_state(6, 5208)
    circ = q.Circuit.from_problem(pr)
    ctx.set_option(q.OPT_METRIC_KIND, 1)
    try:
        G, _ = ctx.metric(circ, pr.theta, in_state=pr.in_state)
    finally:
        ctx.set_option(q.OPT_METRIC_KIND, 0)
    state = pr.in_state.copy()
    idx = np.arange(1 << pr.n_qubits)
    worst = 0.0
    for g in pr.gates:
        kind, q0, _, p = (int(v) for v in g)
        if p >= 0:
            want = 0.25 * float(np.sum(np.abs(state[(idx >> q0) & 1 == 1]) ** 2)) if kind >= W.CRX else 0.25
            worst = max(worst, abs(G[p, p] - want))
        state = oracle.apply_gate(pr.n_qubits, g, pr.theta, state)
    say(f"diagonal: max |L_ii - want| = {worst:.2e}")
    assert worst <= 1e-12


@pytest.mark.parametrize("n,layers", [(4, 3), (9, 2), (13, 2)])
def test_controlled_ring_ansatz(env, n, layers):
    torch, q, ctx = env
    pr = W.controlled_layers(n, layers, 9, 5210 + n)
    say(f"case: {pr.name}")
    res = ctx.step(q.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov)
    check(res, oracle.step(pr), pr, TOL, pr.name)


def test_controlled_complex64_bound(env):
    torch, q, ctx = env
    pr = W.controlled_layers(12, 2, 9, 5220)
    res = ctx.step(q.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov, prec="c64")
    want = oracle.step(pr)
    bound = 4 * pr.n_gates * 2.0 ** -24
    eG, eg = rel_err(res["G"], want["G"]), rel_err(res["grad"], want["grad"])
    eE = abs(res["E"] - want["E"]) / max(1.0, abs(want["E"]))
    say(f"c64 controlled: |dG|={eG:.2e} |dgrad|={eg:.2e} |dE|={eE:.2e} (bound {bound:.1e})")
    assert eG <= bound and eg <= bound and eE <= bound


def test_controlled_shared_angles(env):
    torch, q, ctx = env
    pr = W.share_params(W.controlled_circuit(8, 50, 5230, n_terms=6), 8, 5231)
    say(f"case: controlled with shared angles (P={pr.n_params}, rotations={(pr.gates[:, 3] >= 0).sum()})")
    res = ctx.step(q.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov)
    check(res, oracle.step(pr), pr, TOL, "controlled shared")


@pytest.mark.parametrize("kind", ["block", "l_only"])
def test_controlled_metric_variants(env, kind):
    torch, q, ctx = env
    pr = W.controlled_layers(7, 3, 6, 5240)
    circ = q.Circuit.from_problem(pr)
    blocks = np.repeat(np.arange(3), pr.n_params // 3).astype(np.int32)
    if kind == "block":
        ctx.set_metric_blocks(blocks)
    else:
        ctx.set_option(q.OPT_METRIC_KIND, 1)
    try:
        G, T = ctx.metric(circ, pr.theta)
    finally:
        ctx.set_metric_blocks(None)
        ctx.set_option(q.OPT_METRIC_KIND, 0)
    Go, To = oracle.metric(pr)
    if kind == "block":
        want = np.where(blocks[:, None] == blocks[None, :], Go, 0.0)
    else:
        D, _ = oracle.derivative_states(pr)
        want = D.conj() @ D.T
    eG, eT = rel_err(G, want), rel_err(T, To)
    say(f"{kind}: |dG|={eG:.2e} |dT|={eT:.2e}")
    assert eG <= TOL and eT <= TOL


def test_controlled_device_entry_points(env):
    """apply_circuit_dev (forward state), metric_dev and the autograd energy."""
    torch, q, ctx = env
    from paper_2011_02991_amd import torch_energy as te
    pr = W.controlled_circuit(8, 60, 5250, n_terms=7)
    pr.in_state = W.random_state(8, 5251)
    circ = q.Circuit.from_problem(pr)
    st = torch.as_tensor(pr.in_state, dtype=torch.complex128).cuda().contiguous()
    ctx.apply_circuit_dev(circ, pr.theta, st.data_ptr())
    torch.cuda.synchronize()
    ef = rel_err(st.cpu().numpy(), oracle.forward(pr))
    Gd = torch.zeros((pr.n_params, pr.n_params), dtype=torch.complex128, device="cuda")
    Td = torch.zeros(pr.n_params, dtype=torch.complex128, device="cuda")
    ins = torch.as_tensor(pr.in_state, dtype=torch.complex128).cuda().contiguous()
    ctx.metric_dev(circ, pr.theta, Gd.data_ptr(), Td.data_ptr(), in_state_dev_ptr=ins.data_ptr())
    torch.cuda.synchronize()
    Go, To = oracle.metric(pr)
    eG, eT = rel_err(Gd.cpu().numpy(), Go), rel_err(Td.cpu().numpy(), To)
    th = torch.tensor(pr.theta, dtype=torch.float64, requires_grad=True)
    E = te.energy(ctx, circ, th, in_state=ins)
    E.backward()
    Eo, go = oracle.energy_grad(pr)
    eg = rel_err(th.grad.numpy(), go)
    say(f"device: |dpsi|={ef:.2e} |dG|={eG:.2e} |dT|={eT:.2e} |dE|={abs(E.item() - Eo):.2e} |dgrad|={eg:.2e}")
    assert ef <= 1e-12 and eG <= TOL and eT <= TOL and eg <= TOL
    assert abs(E.item() - Eo) <= TOL * max(1.0, abs(Eo))


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_controlled_in_batched(env, prec):
    """qng_step_batched with controlled rotations beside plain members: the
    batch's forward registers apply them from the gate table and take their
    diagonals (1/4 Prob(control = 1)) on the way, a column whose top or the
    rotation below it is controlled is seeded on its own with its generator,
    and the sweeps run the kernels with the controlled handlers.  Eager and
    replayed, against the oracle (complex128 at 1e-10, complex64 at the FP32
    rounding bound) and against the single step."""
    torch, q, ctx = env
    probs = [W.scaled(W.config1, 6, 1, seed=5260), W.controlled_layers(5, 1, 4, 5261),
             W.controlled_circuit(7, 40, 5262, n_terms=5), W.controlled_layers(12, 2, 6, 5263),
             W.controlled_circuit(3, 14, 5264, n_terms=3), W.controlled_layers(2, 2, 3, 5265)]
    probs[2].in_state = W.random_state(7, 5266)
    circs = [q.Circuit.from_problem(p) for p in probs]
    ths = [p.theta for p in probs]
    for rep in range(2):   # the second call replays the captured graph
        res = ctx.step_batched(circs, ths, 0.1, 1e-4, in_states=[p.in_state for p in probs], prec=prec)
        for b, p in enumerate(probs):
            want = oracle.step(p)
            tol = TOL if prec == "c128" else 8 * np.sqrt(p.n_gates) * 2.0 ** -24
            eG, eg = rel_err(res[b]["G"], want["G"]), rel_err(res[b]["grad"], want["grad"])
            say(f"{prec} rep {rep} member {b} ({p.name}): |dG|={eG:.2e} |dgrad|={eg:.2e}")
            assert eG <= tol and eg <= tol, (b, eG, eg, tol)
            single = ctx.step(circs[b], ths[b], 0.1, 1e-4, in_state=p.in_state, prec=prec)
            assert rel_err(res[b]["G"], single["G"]) <= (1e-12 if prec == "c128" else tol)


@pytest.mark.timeout(600)
def test_controlled_n22_sampled(env):
    """n = 22, two ring layers (P = 88): sampled metric entries and gradient
    entries against the oracle's derivative states of the sampled parameters."""
    torch, q, ctx = env
    pr = W.controlled_layers(22, 2, 30, 5270)
    circ = q.Circuit.from_problem(pr)
    say(f"case: {pr.name} step")
    res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov)
    st = ctx.stats()
    say(f"metric {st['metric_ms']:.0f} ms, grad {st['grad_ms']:.0f} ms, elements {st['elements']}")
    rng = np.random.default_rng(5271)
    sel = np.array(sorted({0, 21, 22, 43, 44, pr.n_params - 1, int(rng.integers(0, pr.n_params))}))
    say(f"oracle derivative states for {list(sel)}")
    D, psi = oracle.derivative_states(pr, sel)
    Go, To, _ = oracle.metric_from_states(D, psi)
    Eo, go = oracle.energy_grad(pr, sel, D=D, psi=psi)
    eG = rel_err(res["G"][np.ix_(sel, sel)], Go)
    eg = rel_err(res["grad"][sel], go)
    eE = abs(res["E"] - Eo) / max(1.0, abs(Eo))
    say(f"n22: |dG|={eG:.2e} |dgrad|={eg:.2e} |dE|={eE:.2e}")
    assert eG <= TOL and eg <= TOL and eE <= TOL
    # Re G symmetric, diagonal = 1/4 or 1/4 Prob(control) - |T|^2 >= 0
    assert np.allclose(res["G"], res["G"].conj().T, atol=1e-14)
    assert (np.diag(res["G"]).real >= -1e-14).all()


FUSED_CASES = [
    ("ring n13", lambda: W.controlled_layers(13, 2, 6, 5290)),
    # from |0...0> a random list can leave E and grad E at rounding level: an input state
    ("random n14 in-state", lambda: W.controlled_circuit(14, 90, 5291, controlled_fraction=0.5, n_terms=6)),
    ("random n16 in-state", lambda: W.controlled_circuit(16, 70, 5292, n_terms=6)),
    ("ring n15 shared", lambda: W.share_params(W.controlled_layers(15, 2, 6, 5293), 25, 5294)),
]


@pytest.mark.parametrize("label,make", FUSED_CASES, ids=[c[0] for c in FUSED_CASES])
def test_controlled_fused_matches_per_primitive_kernels(env, label, make):
    """The fused passes against the per-primitive kernels (fusion off) on the
    same inputs, and against the oracle: complex128 with one and two columns
    per sweep; complex64 with FP32 shares and with exact FP64 products (each
    against the oracle at the storage bound); the step's real-part products."""
    torch, q, ctx = env
    pr = make()
    if "in-state" in label:
        pr.in_state = W.random_state(pr.n_qubits, 5295)
    circ = q.Circuit.from_problem(pr)
    say(f"case: {pr.name} ({label}, P={pr.n_params}, M={pr.n_gates})")
    want = oracle.step(pr)
    ctx.set_option(q.OPT_FUSION, 0)
    try:
        ref = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
        Gref, Tref = ctx.metric(circ, pr.theta, in_state=pr.in_state)
    finally:
        ctx.set_option(q.OPT_FUSION, 1)
    check(ref, want, pr, TOL, label + " per-primitive")
    for block in (1, 2):
        ctx.set_option(q.OPT_BLOCK_COLUMNS, block)
        try:
            res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
            st = ctx.stats()
            G, T = ctx.metric(circ, pr.theta, in_state=pr.in_state)
        finally:
            ctx.set_option(q.OPT_BLOCK_COLUMNS, 0)
        assert st["sweep_launches"] > 0 and st["block_columns"] == block
        eG, eT = rel_err(G, Gref), rel_err(T, Tref)
        eg = rel_err(res["grad"], ref["grad"])
        say(f"fused (block {block}) vs per-primitive: |dG|={eG:.2e} |dT|={eT:.2e} |dgrad|={eg:.2e}")
        assert eG <= 1e-12 and eT <= 1e-12 and eg <= 1e-12
        check(res, want, pr, TOL, f"{label} fused block {block}")
    bound = 4 * pr.n_gates * 2.0 ** -24
    for exact in (1, 0):
        ctx.set_option(q.OPT_EXACT_PRODUCTS, exact)
        try:
            r64 = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state, prec="c64")
            assert ctx.stats()["sweep_launches"] > 0
            G64, T64 = ctx.metric(circ, pr.theta, in_state=pr.in_state, prec="c64")
        finally:
            ctx.set_option(q.OPT_EXACT_PRODUCTS, 1)
        eG, eT, eg = rel_err(G64, want["G"]), rel_err(T64, Tref), rel_err(r64["grad"], want["grad"])
        say(f"c64 fused (exact products {exact}): |dG|={eG:.2e} |dT|={eT:.2e} |dgrad|={eg:.2e} bound {bound:.1e}")
        assert eG <= bound and eT <= bound and eg <= bound


@pytest.mark.parametrize("make", [lambda: W.controlled_layers(9, 3, 6, 5280),
                                  lambda: W.string_circuit(10, 61, 5281, n_terms=6),
                                  lambda: W.share_params(W.controlled_circuit(8, 45, 5282), 11, 5283)])
def test_stepped_blocks_match_per_primitive_kernels(env, make):
    """With fusion on, circuits with Pauli-string rotations sweep up to 8
    columns per lambda sweep, one kernel per step (products of every column,
    then the adjoint), and controlled ones run on the fused passes; with fusion
    off, one kernel per primitive.  P is not a multiple of 8, so the last
    block of a stepped sweep is ragged.  Both against each other and against
    the oracle."""
    torch, q, ctx = env
    pr = make()
    pr.in_state = W.random_state(pr.n_qubits, 5284)
    circ = q.Circuit.from_problem(pr)
    say(f"case: {pr.name} (P={pr.n_params}, rotations={(pr.gates[:, 3] >= 0).sum()})")
    a = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
    st = ctx.stats()
    ctx.set_option(q.OPT_FUSION, 0)
    try:
        b = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
        st0 = ctx.stats()
    finally:
        ctx.set_option(q.OPT_FUSION, 1)
    say(f"launches: stepped {st['other_launches']}, per primitive {st0['other_launches']}")
    assert st["other_launches"] < st0["other_launches"]
    for key in ("G", "grad"):
        assert rel_err(a[key], b[key]) <= 1e-12, key
    check(a, oracle.step(pr), pr, TOL, pr.name + " stepped")
