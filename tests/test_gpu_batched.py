"""qng_step_batched: many ansaetze of uneven register size and depth swept
together (every sweep launch carries tiles of several ansaetze), with the
metric phase captured into a hipGraph and replayed, and the autotuner.

Every member is compared with the oracle (complex128: 1e-10 normwise, as in
the single-ansatz tests).  For the 64-ansatz workload (n in [12, 22], 2..8
layers of RY, RZ + CNOT chain, 30-term Hamiltonians) each member is compared
with the single-ansatz entry point on every entry, with the full oracle when
n <= 16 and with the oracle on sampled parameters (first, last, one in the
middle) above that.
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
    import torch  # noqa: F401
    import paper_2011_02991_amd as q
    c = q.Context(0)
    yield q, c
    c.close()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300))


def mixed_batch():
    """Members of several register classes (n below and above the tile width),
    including one without parameters and one with a single parameter."""
    out = [W.scaled(W.config1, 12, 2, seed=7001), W.scaled(W.config2, 9, 3, seed=7002),
           W.scaled(W.config3, 13, 1, seed=7003), W.random_circuit(5, 30, 7004, n_terms=4),
           W.scaled(W.config5, 11, 2, seed=7005), W.scaled(W.config1, 12, 3, seed=7006)]
    none = W.random_circuit(4, 6, 7007, fixed_fraction=1.0, n_terms=3)
    one = W.random_circuit(6, 1, 7008, fixed_fraction=0.0, n_terms=3)
    psi = W.random_state(6, 7009)
    one.in_state = psi
    return out + [none, one]


def check_member(res, want, pr, tol, label):
    eG = rel_err(res["G"], want["G"]) if pr.n_params else 0.0
    eg = rel_err(res["grad"], want["grad"]) if pr.n_params else 0.0
    eE = abs(res["E"] - want["E"]) / max(1.0, abs(want["E"]))
    ed = rel_err(res["dtheta"], want["dtheta"]) if pr.n_params else 0.0
    kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(pr.n_params)) if pr.n_params else 1.0
    assert eG <= tol and eg <= tol and eE <= tol, (label, eG, eg, eE)
    assert ed <= max(tol, kappa * 1e-14), (label, ed, kappa)


def run_batch(q, ctx, probs, thetas=None, prec="c128"):
    circs = [q.Circuit.from_problem(p) for p in probs]
    ths = thetas if thetas is not None else [p.theta for p in probs]
    return ctx.step_batched(circs, ths, probs[0].dt, probs[0].tikhonov,
                            in_states=[p.in_state for p in probs], prec=prec)


def test_mixed_batch_vs_oracle(env):
    q, ctx = env
    probs = mixed_batch()
    say(f"case: mixed batch of {len(probs)} ({[(p.n_qubits, p.n_params) for p in probs]})")
    ctx.set_option(q.OPT_GRAPH, 0)
    res = run_batch(q, ctx, probs)
    st = ctx.stats()
    say(f"stats: {st}")
    for b, (r, p) in enumerate(zip(res, probs)):
        check_member(r, oracle.step(p), p, TOL, f"member {b}")
    ctx.set_option(q.OPT_GRAPH, 1)


@pytest.mark.parametrize("graph", [0, 1])
def test_tiny_registers_batch(env, graph):
    """Members of 2, 3 and 4 qubits beside larger ones: the column seeds of a
    launch run as one kernel per round over groups of eight amplitudes, which
    a 3-qubit register fills exactly; a 2-qubit register is seeded on its own.
    Layered members put two rotations on one qubit back to back (the seed's
    rotation on the seeded qubit itself)."""
    q, ctx = env
    probs = [W.random_circuit(2, 12, 7201, n_terms=3), W.random_circuit(3, 16, 7202, n_terms=3),
             W.scaled(W.config2, 3, 2, seed=7203), W.random_circuit(4, 20, 7204, n_terms=4),
             W.scaled(W.config3, 10, 2, seed=7205), W.scaled(W.config2, 2, 3, seed=7206)]
    probs[1].in_state = W.random_state(3, 7207)
    say(f"case: tiny registers batch, graph {graph} ({[(p.n_qubits, p.n_params) for p in probs]})")
    ctx.set_option(q.OPT_GRAPH, graph)
    try:
        for rep in range(2 if graph else 1):
            res = run_batch(q, ctx, probs)
            for b, (r, p) in enumerate(zip(res, probs)):
                check_member(r, oracle.step(p), p, TOL, f"rep {rep} member {b}")
    finally:
        ctx.set_option(q.OPT_GRAPH, 1)


@pytest.mark.parametrize("graph", [0, 1])
def test_complex64_batch(env, graph):
    """complex64 storage (FP32 registers, every product formed in FP64): the
    mixed batch and registers of 2 to 4 qubits, each member against its
    complex128 batch result and the oracle at the random-walk rounding bound of
    its sweeps (8 sqrt(M) u, M gates, u = 2^-24), and against the complex64
    single-ansatz step (the same FP32 arithmetic, other kernels and
    reduction orders: the same bound)."""
    q, ctx = env
    probs = mixed_batch() + [W.random_circuit(2, 12, 7201, n_terms=3), W.random_circuit(3, 16, 7202, n_terms=3),
                             W.random_circuit(4, 20, 7204, n_terms=4)]
    say(f"case: complex64 batch, graph {graph} ({[(p.n_qubits, p.n_params) for p in probs]})")
    ctx.set_option(q.OPT_GRAPH, graph)
    try:
        res = run_batch(q, ctx, probs, prec="c64")
        if graph:
            res = run_batch(q, ctx, probs, prec="c64")   # a replay
        ref = run_batch(q, ctx, probs, prec="c128")
    finally:
        ctx.set_option(q.OPT_GRAPH, 1)
    for b, p in enumerate(probs):
        if not p.n_params:
            continue
        bound = 8 * np.sqrt(p.n_gates) * 2.0 ** -24
        single = ctx.step(q.Circuit.from_problem(p), p.theta, p.dt, p.tikhonov, in_state=p.in_state, prec="c64")
        want = oracle.step(p)
        for key in ("G", "grad"):
            e_ref, e_or = rel_err(res[b][key], ref[b][key]), rel_err(res[b][key], want[key])
            e_single = rel_err(res[b][key], single[key])
            assert e_ref <= bound and e_or <= bound and e_single <= bound, (b, key, e_ref, e_or, e_single, bound)
        assert abs(res[b]["E"] - want["E"]) <= bound * max(1.0, abs(want["E"]))


def test_graph_replays_match_eager(env):
    """The metric phase is captured on the first call and replayed with new
    angles; eager calls and host work run between the replays, and every
    replay is checked against an eager run and the oracle."""
    q, ctx = env
    probs = mixed_batch()[:5]
    rng = np.random.default_rng(31)
    ctx.set_option(q.OPT_GRAPH, 1)
    for rep in range(4):
        thetas = [rng.uniform(0, 2 * np.pi, p.n_params) for p in probs]
        say(f"case: graph replay {rep}")
        got = run_batch(q, ctx, probs, thetas)
        replays = ctx.stats()["graph_replays"]
        ctx.set_option(q.OPT_GRAPH, 0)
        eager = run_batch(q, ctx, probs, thetas)
        ctx.set_option(q.OPT_GRAPH, 1)
        say(f"graph_replays={replays}")
        if rep > 0:
            assert replays > 0
        for b, p in enumerate(probs):
            assert np.array_equal(got[b]["G"], eager[b]["G"]) and np.array_equal(got[b]["grad"], eager[b]["grad"])
            at = W.Problem(**{**p.__dict__, "theta": thetas[b]})
            check_member(got[b], oracle.step(at), at, TOL, f"replay {rep} member {b}")


def test_graph_replay_with_reordered_members(env):
    """The same ansaetze in another order move every member's registers in the
    workspace while each register class keeps its structure key: the captured
    graph of a class must not be replayed with the old member addresses.  The
    batch (members of three register classes) is run in one order and then
    reversed, both through the graph, and every member is checked against an
    eager run of the same order and the oracle."""
    q, ctx = env
    base = [W.scaled(W.config1, 9, 2, seed=7101), W.scaled(W.config3, 12, 2, seed=7102),
            W.scaled(W.config2, 13, 1, seed=7103), W.scaled(W.config5, 10, 1, seed=7104)]
    ctx.set_option(q.OPT_GRAPH, 1)
    for order in (base, base[::-1], base, base[::-1]):
        say(f"case: reordered batch {[p.n_qubits for p in order]}")
        got = run_batch(q, ctx, order)
        ctx.set_option(q.OPT_GRAPH, 0)
        eager = run_batch(q, ctx, order)
        ctx.set_option(q.OPT_GRAPH, 1)
        for b, p in enumerate(order):
            assert np.array_equal(got[b]["G"], eager[b]["G"]) and np.array_equal(got[b]["grad"], eager[b]["grad"])
            check_member(got[b], oracle.step(p), p, TOL, f"order {[x.n_qubits for x in order]} member {b}")


def test_autotuner(env):
    q, ctx = env
    probs = mixed_batch()[:3]
    ctx.set_option(q.OPT_AUTOTUNE, 1)
    try:
        say("case: autotune first call")
        r1 = run_batch(q, ctx, probs)
        s1 = ctx.stats()
        say(f"tuned: tile {s1['tile_qubits']}, target {s1['target_tiles']}, {s1['tune_ms']:.1f} ms")
        assert s1["tune_ms"] > 0
        assert s1["tile_qubits"] in (10, 11, 12) and s1["target_tiles"] in (2048, 4096, 8192)
        r2 = run_batch(q, ctx, probs)
        s2 = ctx.stats()
        assert s2["tune_ms"] == 0 and s2["tile_qubits"] == s1["tile_qubits"]
        for b, p in enumerate(probs):
            want = oracle.step(p)
            check_member(r1[b], want, p, TOL, f"tuned member {b}")
            check_member(r2[b], want, p, TOL, f"tuned member {b} (cached)")
    finally:
        ctx.set_option(q.OPT_AUTOTUNE, 0)


@pytest.mark.timeout(1100)
def test_64_ansatz_workload(env):
    q, ctx = env
    probs = W.config4()
    say(f"case: 64-ansatz batch, n {min(p.n_qubits for p in probs)}..{max(p.n_qubits for p in probs)}, "
        f"P {min(p.n_params for p in probs)}..{max(p.n_params for p in probs)}")
    import time
    t0 = time.perf_counter()
    res = run_batch(q, ctx, probs)
    t1 = time.perf_counter()
    res2 = run_batch(q, ctx, probs)      # graph replay
    t2 = time.perf_counter()
    st = ctx.stats()
    say(f"batched: first call {t1 - t0:.2f} s, replay {t2 - t1:.2f} s; launches {st['sweep_launches']}, "
        f"graph_replays {st['graph_replays']}")
    single = []
    t3 = time.perf_counter()
    for p in probs:
        single.append(ctx.step(q.Circuit.from_problem(p), p.theta, p.dt, p.tikhonov))
    t4 = time.perf_counter()
    say(f"one call per ansatz: {t4 - t3:.2f} s")
    worst = 0.0
    for b, p in enumerate(probs):
        for key in ("G", "grad", "dtheta"):
            e = rel_err(res2[b][key], single[b][key])
            worst = max(worst, e)
            assert e <= 1e-12 or key == "dtheta", (b, key, e)
        assert abs(res2[b]["E"] - single[b]["E"]) <= 1e-12 * max(1.0, abs(single[b]["E"]))
        assert np.array_equal(res[b]["G"], res2[b]["G"])
    say(f"batched vs single: worst {worst:.2e}")
    say("oracle on every parameter of the members with n <= 16, on sampled parameters of the others")
    for b, p in enumerate(probs):
        if p.n_qubits <= 16:
            want = oracle.step(p)
            check_member(res2[b], want, p, TOL, f"member {b} (n={p.n_qubits}, P={p.n_params}, full oracle)")
            continue
        sel = np.array([0, p.n_params // 2, p.n_params - 1])
        D, psi = oracle.derivative_states(p, sel)
        Go, To, _ = oracle.metric_from_states(D, psi)
        Eo, go = oracle.energy_grad(p, sel, D=D, psi=psi)
        del D, psi
        eG = rel_err(res2[b]["G"][np.ix_(sel, sel)], Go)
        eg = rel_err(res2[b]["grad"][sel], go)
        eE = abs(res2[b]["E"] - Eo) / max(1.0, abs(Eo))
        assert eG <= TOL and eg <= TOL and eE <= TOL, (b, eG, eg, eE)
        if b % 8 == 0:
            say(f"member {b} (n={p.n_qubits}, P={p.n_params}): |dG|={eG:.2e} |dgrad|={eg:.2e} |dE|={eE:.2e}")


def test_batch_without_G_outputs(env):
    """Without G outputs the batched sweeps keep the real parts of the metric's
    inner products (the solves read Re G only): the same dtheta, gradient and
    energy as with the G outputs, through eager runs and graph replays."""
    q, ctx = env
    probs = mixed_batch()[:6]
    circs = [q.Circuit.from_problem(p) for p in probs]
    ths = [p.theta for p in probs]
    ins = [p.in_state for p in probs]
    full = ctx.step_batched(circs, ths, probs[0].dt, probs[0].tikhonov, in_states=ins, want_G=True)
    for rep in range(2):
        real = ctx.step_batched(circs, ths, probs[0].dt, probs[0].tikhonov, in_states=ins, want_G=False)
        for b, p in enumerate(probs):
            if not p.n_params:
                continue
            ed = rel_err(real[b]["dtheta"], full[b]["dtheta"])
            assert ed <= 1e-13, (rep, b, ed)
            assert np.array_equal(real[b]["grad"], full[b]["grad"]) and real[b]["E"] == full[b]["E"]
    say(f"replays {ctx.stats()['graph_replays']}")


def test_small_register_batch_pays(env):
    """Batches of small registers (n <= 16), where one ansatz alone cannot fill
    the GPU: 48 ansaetze of n in [8, 16], 2..6 layers, batched (graph replay)
    against one qng_step per ansatz; every member against the oracle."""
    import time
    q, ctx = env
    rng = np.random.default_rng(7201)
    probs = [W.make_problem(f"small{b}", int(rng.integers(8, 17)), int(rng.integers(2, 7)), (W.RY, W.RZ),
                            "cnot_chain", 12, 7300 + b) for b in range(48)]
    circs = [q.Circuit.from_problem(p) for p in probs]
    ths = [p.theta for p in probs]
    ctx.set_option(q.OPT_GRAPH, 1)
    run_batch(q, ctx, probs)                  # builds and captures
    ctx.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        res = ctx.step_batched(circs, ths, probs[0].dt, probs[0].tikhonov, want_G=False)
    t1 = time.perf_counter()
    for _ in range(reps):
        single = [ctx.step(c, t, p.dt, p.tikhonov, want_G=False) for c, t, p in zip(circs, ths, probs)]
    t2 = time.perf_counter()
    say(f"48 small ansaetze: batched {(t1 - t0) / reps * 1e3:.1f} ms per step of all, "
        f"one call per ansatz {(t2 - t1) / reps * 1e3:.1f} ms")
    for b, p in enumerate(probs):
        want = oracle.step(p)
        kappa = np.linalg.cond(want["G"].real + p.tikhonov * np.eye(p.n_params))
        assert rel_err(res[b]["grad"], want["grad"]) <= TOL
        assert rel_err(res[b]["dtheta"], want["dtheta"]) <= max(TOL, kappa * 1e-14)
        assert rel_err(res[b]["dtheta"], single[b]["dtheta"]) <= max(1e-12, kappa * 1e-14)
