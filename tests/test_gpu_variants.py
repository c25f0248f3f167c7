"""Cheaper metric variants against the FP64 CPU oracle: the block-diagonal
approximation (entries between parameters of one block only; every column's
sweep stops at the lowest rotation of its block) and the L-only matrix
(G without the conj(T_i) T_j term).

References: the oracle's G from the definition with the entries between
different blocks set to zero, and its L = <d_i psi, d_j psi> (the Gram matrix of
the derivative states).  Tolerance 1e-10 normwise (complex128) as for the full
metric; the natural-gradient step with a block-diagonal G is checked against
the solve of the oracle's masked G.
"""
import sys
import time

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


def layer_blocks(pr, layers):
    return np.repeat(np.arange(layers), pr.n_params // layers).astype(np.int32)


def masked(G, blocks):
    return np.where(blocks[:, None] == blocks[None, :], G, 0.0)


@pytest.mark.parametrize("fusion", [1, 0])
@pytest.mark.parametrize("label,make,layers", [
    ("cfg3 n=10 L=3", lambda: W.scaled(W.config3, 10, 3, n_terms=8), 3),
    ("cfg2 n=13 L=2", lambda: W.scaled(W.config2, 13, 2, n_terms=8), 2),
])
def test_block_diagonal_per_layer(env, fusion, label, make, layers):
    q, ctx = env
    pr = make()
    blocks = layer_blocks(pr, layers)
    say(f"case: {label} block-diagonal per layer, fusion={fusion}")
    circ = q.Circuit.from_problem(pr)
    ctx.set_option(q.OPT_FUSION, fusion)
    ctx.set_metric_blocks(blocks)
    try:
        G, T = ctx.metric(circ, pr.theta)
        res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov)
        st = ctx.stats()
    finally:
        ctx.set_metric_blocks(None)
        ctx.set_option(q.OPT_FUSION, 1)
    Gw, Tw = oracle.metric(pr)
    Gb = masked(Gw, blocks)
    eG, eT = rel_err(G, Gb), rel_err(T, Tw)
    want = oracle.step(pr)
    dth = oracle.solve_step(Gb, want["grad"], pr.dt, pr.tikhonov)
    ed = rel_err(res["dtheta"], dth)
    kappa = np.linalg.cond(Gb.real + pr.tikhonov * np.eye(pr.n_params))
    say(f"  |dG|={eG:.2e} |dT|={eT:.2e} |ddtheta|={ed:.2e} kappa={kappa:.1e} elements={st['elements']}")
    assert eG <= TOL and eT <= TOL
    assert rel_err(res["G"], Gb) <= TOL and rel_err(res["grad"], want["grad"]) <= TOL
    assert ed <= max(TOL, kappa * 1e-14)
    assert np.all(G[blocks[:, None] != blocks[None, :]] == 0)


def test_block_diagonal_irregular_blocks_shared_params(env):
    """Blocks that are not contiguous in gate order, on a circuit whose
    parameters are shared by several rotations."""
    q, ctx = env
    pr = W.share_params(W.random_circuit(9, 60, 5101, n_terms=6), 12, 5102)
    pr.in_state = W.random_state(9, 5103)
    blocks = (np.arange(pr.n_params) % 3).astype(np.int32)
    ctx.set_metric_blocks(blocks)
    try:
        G, T = ctx.metric(q.Circuit.from_problem(pr), pr.theta, in_state=pr.in_state)
    finally:
        ctx.set_metric_blocks(None)
    Gw, Tw = oracle.metric(pr)
    eG = rel_err(G, masked(Gw, blocks))
    say(f"irregular blocks, shared parameters: |dG|={eG:.2e}")
    assert eG <= TOL and rel_err(T, Tw) <= TOL


@pytest.mark.parametrize("label,make", [
    ("cfg1 n=8", lambda: W.scaled(W.config1, 8, 2, n_terms=6)),
    ("random n=12", lambda: W.random_circuit(12, 50, 5104, n_terms=6)),
])
def test_l_only(env, label, make):
    q, ctx = env
    pr = make()
    ctx.set_option(q.OPT_METRIC_KIND, 1)
    try:
        L, T = ctx.metric(q.Circuit.from_problem(pr), pr.theta)
    finally:
        ctx.set_option(q.OPT_METRIC_KIND, 0)
    D, psi = oracle.derivative_states(pr)
    _, To, Lo = oracle.metric_from_states(D, psi)
    eL = rel_err(L, Lo)
    say(f"{label} L only: |dL|={eL:.2e}")
    assert eL <= TOL and rel_err(T, To) <= TOL


def test_block_diagonal_is_cheaper_at_n20(env):
    """Per-layer blocks at n=20, 4 layers: a quarter of the elements; the
    sampled entries inside the blocks match the oracle."""
    q, ctx = env
    pr = W.scaled(W.config3, 20, 4, n_terms=10)
    circ = q.Circuit.from_problem(pr)
    blocks = layer_blocks(pr, 4)
    ctx.metric(circ, pr.theta)                     # warm-up (plans, workspace)
    t0 = time.perf_counter()
    Gf, _ = ctx.metric(circ, pr.theta)
    t1 = time.perf_counter()
    ctx.set_metric_blocks(blocks)
    try:
        ctx.metric(circ, pr.theta)
        t2 = time.perf_counter()
        Gb, _ = ctx.metric(circ, pr.theta)
        t3 = time.perf_counter()
    finally:
        ctx.set_metric_blocks(None)
    say(f"n=20 P={pr.n_params}: full {1e3 * (t1 - t0):.1f} ms, block-diagonal {1e3 * (t3 - t2):.1f} ms")
    np.testing.assert_allclose(Gb, masked(Gf, blocks), atol=1e-12 * np.abs(Gf).max())
    sel = np.array([0, 1, 37, 38, pr.n_params - 2, pr.n_params - 1])
    Go, _ = oracle.metric(pr, sel)
    want = masked(Go, blocks[sel])
    assert rel_err(Gb[np.ix_(sel, sel)], want) <= TOL


def test_settings_errors(env):
    q, ctx = env
    pr = W.scaled(W.config1, 5, 1)
    ctx.set_metric_blocks(np.zeros(pr.n_params + 1, dtype=np.int32))
    try:
        with pytest.raises(q.QNGError) as e:
            ctx.metric(q.Circuit.from_problem(pr), pr.theta)
        assert e.value.name == "QNG_E_INVALID_ARG"
        with pytest.raises(q.QNGError):
            ctx.step_batched([q.Circuit.from_problem(pr)], [pr.theta], 0.1, 1e-4)
    finally:
        ctx.set_metric_blocks(None)
    with pytest.raises(q.QNGError):
        ctx.set_option(q.OPT_METRIC_KIND, 2)


@pytest.mark.parametrize("variant", ["blocks", "l_only", "shared"])
def test_step_without_G_output_in_variants(env, variant):
    """The real-part passes of a step without a G output under the cheaper
    variants and shared parameters: the same dtheta as the step that returns G."""
    q, ctx = env
    pr = W.scaled(W.config3, 13, 3, n_terms=8)
    if variant == "shared":
        pr = W.share_params(pr, 30, 771)
    circ = q.Circuit.from_problem(pr)
    if variant == "blocks":
        ctx.set_metric_blocks(layer_blocks(pr, 3))
    elif variant == "l_only":
        ctx.set_option(q.OPT_METRIC_KIND, 1)
    try:
        full = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, want_G=True)
        real = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, want_G=False)
    finally:
        ctx.set_metric_blocks(None)
        ctx.set_option(q.OPT_METRIC_KIND, 0)
    ed = rel_err(real["dtheta"], full["dtheta"])
    say(f"{variant}: |ddtheta| real vs full {ed:.2e}")
    assert ed <= 1e-13
