"""Pauli-string rotations exp(i theta S/2) against the FP64 CPU oracle.

The column of a Pauli-string rotation uses the string S itself as generator
(seed phi = S y, products <lambda|S|phi>), and S^2 = 1 keeps the diagonal at
1/4 (Sec. 2).  With fusion on, the library rewrites every string rotation as
basis rotations, CNOTs onto the string's lowest qubit and an RZ there carrying
the parameter (the same unitary), and the fused passes take the circuit; with
fusion off, the per-primitive string kernels run.  complex128 results must
match the oracle to 1e-10 normwise (Delta theta: kappa(Re G + eps I) * 1e-14
when larger), and the two routes each other to 1e-12; complex64 the oracle to
4 M' 2^-24 with M' the gates of the rewritten list.

Workloads: random circuits with strings of 1..4 letters among plain
rotations, CNOT and CZ (n = 2 .. 14, input states, permuted parameters); the
layered ansatz of RX, ZZ ladders and an X Y..Y X string; strings together with
controlled rotations and shared angles; the L-only variant; the device entry
points with the autograd energy; n = 22 sampled entries; both routes with one
and two columns per sweep, FP32 shares and exact products, and the
derivative-state variant.
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


def combined(n, seed):
    """A string circuit followed by a controlled-rotation circuit on the same
    register (parameters of the second numbered after the first's)."""
    a = W.string_circuit(n, 30, seed, n_terms=6)
    b = W.controlled_circuit(n, 30, seed + 1)
    gb = b.gates.copy()
    gb[gb[:, 3] >= 0, 3] += a.n_params
    return W.Problem(name=f"strings+controlled_n{n}", n_qubits=n, gates=np.concatenate([a.gates, gb]),
                     theta=np.concatenate([a.theta, b.theta]), pauli=a.pauli, coeff=a.coeff, strings=a.strings)


def rewritten_gates(pr):
    """Gates of the rewritten list: a string of k letters, x of them X or Y,
    becomes 2 x basis rotations, 2 (k - 1) CNOTs and one RZ."""
    m = 0
    for g in pr.gates:
        if int(g[0]) != W.RPAULI:
            m += 1
            continue
        letters = pr.strings[int(g[1])]
        k, x = int((letters > 0).sum()), int(((letters == 1) | (letters == 2)).sum())
        m += 2 * x + 2 * (k - 1) + 1
    return m


CASES = [(2, 12, 5301), (3, 24, 5302), (5, 40, 5303), (7, 60, 5304), (10, 70, 5305), (14, 50, 5306)]


@pytest.mark.parametrize("n,ngates,seed", CASES)
def test_random_string_circuits(env, n, ngates, seed):
    torch, q, ctx = env
    pr = W.string_circuit(n, ngates, seed, n_terms=7)
    if seed % 2 == 0:
        pr.in_state = W.random_state(n, seed)
    if seed % 3 == 0:
        pr = W.permute_params(pr, seed)
    ns = int((pr.gates[:, 0] == W.RPAULI).sum())
    say(f"case: {pr.name} ({ns} string rotations)")
    assert ns > 0
    circ = q.Circuit.from_problem(pr)
    res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
    assert ctx.stats()["sweep_launches"] > 0 or pr.n_params < 2
    want = oracle.step(pr)
    check(res, want, pr, TOL, pr.name)
    G, T = ctx.metric(circ, pr.theta, in_state=pr.in_state)
    assert rel_err(G, want["G"]) <= TOL and rel_err(T, want["T"]) <= TOL


@pytest.mark.parametrize("n,layers", [(2, 2), (6, 3), (12, 2)])
def test_string_layers(env, n, layers):
    torch, q, ctx = env
    pr = W.string_layers(n, layers, 9, 5310 + n)
    say(f"case: {pr.name}")
    res = ctx.step(q.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov)
    check(res, oracle.step(pr), pr, TOL, pr.name)


def test_strings_complex64_bound(env):
    torch, q, ctx = env
    pr = W.string_layers(12, 2, 9, 5320)
    want = oracle.step(pr)
    bound = 4 * rewritten_gates(pr) * 2.0 ** -24
    for fusion in (1, 0):
        ctx.set_option(q.OPT_FUSION, fusion)
        try:
            res = ctx.step(q.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov, prec="c64")
        finally:
            ctx.set_option(q.OPT_FUSION, 1)
        eG, eg = rel_err(res["G"], want["G"]), rel_err(res["grad"], want["grad"])
        eE = abs(res["E"] - want["E"]) / max(1.0, abs(want["E"]))
        say(f"c64 strings (fusion {fusion}): |dG|={eG:.2e} |dgrad|={eg:.2e} |dE|={eE:.2e} (bound {bound:.1e})")
        assert eG <= bound and eg <= bound and eE <= bound


def test_strings_with_controlled_rotations_and_shared_angles(env):
    torch, q, ctx = env
    pr = combined(7, 5330)
    pr.in_state = W.random_state(7, 5331)
    say(f"case: {pr.name} (P={pr.n_params})")
    res = ctx.step(q.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
    check(res, oracle.step(pr), pr, TOL, pr.name)
    sh = W.share_params(pr, 9, 5332)
    res = ctx.step(q.Circuit.from_problem(sh), sh.theta, sh.dt, sh.tikhonov, in_state=sh.in_state)
    check(res, oracle.step(sh), sh, TOL, sh.name + " shared")


def test_strings_l_only(env):
    torch, q, ctx = env
    pr = W.string_layers(6, 2, 6, 5340)
    ctx.set_option(q.OPT_METRIC_KIND, 1)
    try:
        G, T = ctx.metric(q.Circuit.from_problem(pr), pr.theta)
    finally:
        ctx.set_option(q.OPT_METRIC_KIND, 0)
    D, psi = oracle.derivative_states(pr)
    _, To, L = oracle.metric_from_states(D, psi)
    eG, eT = rel_err(G, L), rel_err(T, To)
    say(f"l_only strings: |dL|={eG:.2e} |dT|={eT:.2e}")
    assert eG <= TOL and eT <= TOL
    assert np.allclose(np.diag(G).real, 0.25, atol=1e-14)


def test_strings_device_entry_points(env):
    torch, q, ctx = env
    from paper_2011_02991_amd import torch_energy as te
    pr = W.string_circuit(8, 60, 5350, n_terms=7)
    pr.in_state = W.random_state(8, 5351)
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
def test_strings_in_batched(env, prec):
    """qng_step_batched rewrites Pauli-string rotations as the single step does
    (fixed basis rotations from the circuit's forward table, the passes' fixed
    shears): members with strings beside plain ones, eager and replayed,
    against the oracle (complex128 at 1e-10, complex64 at the FP32 rounding
    bound of the rewritten gate count) and against the single step; a string
    with no letter is rejected."""
    torch, q, ctx = env
    probs = [W.scaled(W.config1, 6, 1, seed=5360), W.string_layers(5, 1, 4, 5361),
             W.string_circuit(7, 40, 5362, n_terms=5), W.string_layers(12, 1, 6, 5363),
             W.string_circuit(3, 12, 5364, n_terms=3)]
    circs = [q.Circuit.from_problem(p) for p in probs]
    ths = [p.theta for p in probs]
    for rep in range(2):   # the second call replays the captured graph
        res = ctx.step_batched(circs, ths, 0.1, 1e-4, prec=prec)
        for b, p in enumerate(probs):
            want = oracle.step(p)
            tol = TOL if prec == "c128" else 8 * np.sqrt(4 * p.n_gates) * 2.0 ** -24
            eG, eg = rel_err(res[b]["G"], want["G"]), rel_err(res[b]["grad"], want["grad"])
            say(f"{prec} rep {rep} member {b} ({p.name}): |dG|={eG:.2e} |dgrad|={eg:.2e}")
            assert eG <= tol and eg <= tol, (b, eG, eg, tol)
            single = ctx.step(circs[b], ths[b], 0.1, 1e-4, prec=prec)
            assert rel_err(res[b]["G"], single["G"]) <= (1e-12 if prec == "c128" else tol)
    # a string with no letter (a global phase) is not rewritten
    bad = W.string_circuit(9, 50, 5390, n_terms=6)
    bad.strings = bad.strings.copy()
    bad.strings[0, :] = 0
    with pytest.raises(q.QNGError) as e:
        ctx.step_batched([q.Circuit.from_problem(probs[0]), q.Circuit.from_problem(bad)],
                         [probs[0].theta, bad.theta], 0.1, 1e-4)
    assert e.value.name == "QNG_E_UNSUPPORTED"


@pytest.mark.timeout(600)
def test_strings_n22_sampled(env):
    """n = 22, two layers (P = 88): sampled metric and gradient entries against
    the oracle's derivative states of the sampled parameters."""
    torch, q, ctx = env
    pr = W.string_layers(22, 2, 30, 5370)
    circ = q.Circuit.from_problem(pr)
    say(f"case: {pr.name} step")
    res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov)
    st = ctx.stats()
    say(f"metric {st['metric_ms']:.0f} ms, grad {st['grad_ms']:.0f} ms, elements {st['elements']}")
    sel = np.array([0, 21, 22, 43, 44, 65, pr.n_params - 1])
    say(f"oracle derivative states for {list(sel)}")
    D, psi = oracle.derivative_states(pr, sel)
    Go, To, _ = oracle.metric_from_states(D, psi)
    Eo, go = oracle.energy_grad(pr, sel, D=D, psi=psi)
    eG = rel_err(res["G"][np.ix_(sel, sel)], Go)
    eg = rel_err(res["grad"][sel], go)
    eE = abs(res["E"] - Eo) / max(1.0, abs(Eo))
    say(f"n22 strings: |dG|={eG:.2e} |dgrad|={eg:.2e} |dE|={eE:.2e}")
    assert eG <= TOL and eg <= TOL and eE <= TOL


FUSED_CASES = [
    ("layers n13", lambda: W.string_layers(13, 2, 6, 5380)),
    ("random n14 in-state", lambda: W.string_circuit(14, 90, 5381, string_fraction=0.5, max_support=6, n_terms=6)),
    ("strings+controlled n12 in-state", lambda: combined(12, 5382)),
    ("layers n15 shared", lambda: W.share_params(W.string_layers(15, 2, 6, 5383), 30, 5384)),
]


@pytest.mark.parametrize("label,make", FUSED_CASES, ids=[c[0] for c in FUSED_CASES])
def test_rewritten_strings_on_fused_passes(env, label, make):
    """The rewritten circuit on the fused passes against the string kernels
    (fusion off) and the oracle: complex128 with one and two columns per
    sweep; complex64 with exact FP64 products and with FP32 shares; the
    derivative-state variant where the circuit has no controlled rotation."""
    torch, q, ctx = env
    pr = make()
    if "in-state" in label:
        pr.in_state = W.random_state(pr.n_qubits, 5385)
    circ = q.Circuit.from_problem(pr)
    say(f"case: {pr.name} ({label}, P={pr.n_params}, M={pr.n_gates}, rewritten {rewritten_gates(pr)})")
    want = oracle.step(pr)
    ctx.set_option(q.OPT_FUSION, 0)
    try:
        ref = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
        Gref, Tref = ctx.metric(circ, pr.theta, in_state=pr.in_state)
    finally:
        ctx.set_option(q.OPT_FUSION, 1)
    check(ref, want, pr, TOL, label + " string kernels")
    for block in (1, 2):
        ctx.set_option(q.OPT_BLOCK_COLUMNS, block)
        try:
            res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
            st = ctx.stats()
            G, T = ctx.metric(circ, pr.theta, in_state=pr.in_state)
        finally:
            ctx.set_option(q.OPT_BLOCK_COLUMNS, 0)
        assert st["sweep_launches"] > 0 and st["block_columns"] == block
        eG, eT, eg = rel_err(G, Gref), rel_err(T, Tref), rel_err(res["grad"], ref["grad"])
        say(f"fused (block {block}) vs string kernels: |dG|={eG:.2e} |dT|={eT:.2e} |dgrad|={eg:.2e}")
        assert eG <= 1e-12 and eT <= 1e-12 and eg <= 1e-12
        check(res, want, pr, TOL, f"{label} fused block {block}")
    bound = 4 * rewritten_gates(pr) * 2.0 ** -24
    for exact in (1, 0):
        ctx.set_option(q.OPT_EXACT_PRODUCTS, exact)
        try:
            r64 = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state, prec="c64")
            assert ctx.stats()["sweep_launches"] > 0
        finally:
            ctx.set_option(q.OPT_EXACT_PRODUCTS, 1)
        eG, eg = rel_err(r64["G"], want["G"]), rel_err(r64["grad"], want["grad"])
        say(f"c64 fused (exact products {exact}): |dG|={eG:.2e} |dgrad|={eg:.2e} bound {bound:.1e}")
        assert eG <= bound and eg <= bound
    if "controlled" in label:
        return
    ctx.set_option(q.OPT_METHOD, 1)
    try:
        rs = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
    finally:
        ctx.set_option(q.OPT_METHOD, 0)
    check(rs, want, pr, TOL, label + " derivative states")


def test_letterless_string_keeps_the_stepped_route(env):
    """A string with no letter (a global phase: its row and column of G are
    zero) cannot be rewritten into gates the fused passes take; such a circuit
    sweeps one kernel per step (no fused sweep launch), several columns per
    lambda sweep, against the oracle."""
    torch, q, ctx = env
    pr = W.string_circuit(9, 50, 5390, n_terms=6)
    assert len(pr.strings) > 1
    pr.strings = pr.strings.copy()
    pr.strings[0, :] = 0
    pr.in_state = W.random_state(9, 5391)
    circ = q.Circuit.from_problem(pr)
    say(f"case: {pr.name} with string 0 the identity (P={pr.n_params})")
    res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state)
    assert ctx.stats()["sweep_launches"] == 0
    want = oracle.step(pr)
    check(res, want, pr, TOL, pr.name + " stepped")
    p0 = int(pr.gates[pr.gates[:, 0] == W.RPAULI][0, 3])
    assert np.abs(res["G"][p0]).max() <= 1e-14 and np.abs(res["G"][:, p0]).max() <= 1e-14
