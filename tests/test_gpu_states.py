"""The derivative-state variant of the metric (QNG_OPT_METHOD = 1): the
appendix's strategy of keeping every derivative state (its last algorithm: each
derivative state prepared from a rolling prefix), here as the same tiled
sweeps without inner products plus one Gram matrix of the P + 1 kept states on
the matrix cores (FP64 products and sums).  Parity against the FP64 oracle
(complex128, normwise 1e-10 for G, T, grad E; dtheta within max(1e-10,
kappa 1e-14)), against the recurrent method on every entry, and on the edge
cases: registers of 2 and 3 qubits (fewer reals per state than one staging
step of the Gram kernel), two parameters, odd P, blocks of one, two and
four columns, permuted and shared parameters, the complex G output (the Gram
matrix's imaginary part) and the step without it; and the same a chunk of
column blocks at a time (chunks forced, and chosen under a memory limit)."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10
U32 = 2.0 ** -24


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


def step(q, ctx, pr, method, prec="c128", want_G=True):
    ctx.set_option(q.OPT_METHOD, method)
    try:
        circ = q.Circuit.from_problem(pr)
        res = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state, prec=prec, want_G=want_G)
        _, T = ctx.metric(circ, pr.theta, in_state=pr.in_state, prec=prec)
    finally:
        ctx.set_option(q.OPT_METHOD, 0)
    return res, T


def small_cases():
    cases = [W.random_circuit(2, 9, 8101, n_terms=3), W.random_circuit(3, 14, 8102, n_terms=4),
             W.random_circuit(2, 2, 8103, fixed_fraction=0.0, n_terms=2),
             W.config1(), W.scaled(W.config2, 9, 3, n_terms=6), W.random_circuit(12, 70, 8104, n_terms=6),
             W.permute_params(W.scaled(W.config3, 13, 2, n_terms=8), 8105),
             W.scaled(W.config5, 14, 1, n_terms=8), W.share_params(W.random_circuit(11, 60, 8106, n_terms=5), 9, 8107)]
    cases[1].in_state = W.random_state(3, 8108)
    cases[5].in_state = W.random_state(12, 8109)
    return cases


@pytest.mark.parametrize("idx", range(9))
def test_states_vs_oracle(env, idx):
    q, ctx = env
    pr = small_cases()[idx]
    say(f"case: {pr.name} n={pr.n_qubits} P={pr.n_params} derivative-state metric vs oracle")
    res, T = step(q, ctx, pr, 1)
    want = oracle.step(pr)
    kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(pr.n_params))
    eG, eT = rel_err(res["G"], want["G"]), rel_err(T, want["T"])
    eg, ed = rel_err(res["grad"], want["grad"]), rel_err(res["dtheta"], want["dtheta"])
    say(f"{pr.name}: |dG|={eG:.2e} |dT|={eT:.2e} |dgrad|={eg:.2e} |ddtheta|={ed:.2e} kappa={kappa:.1e}")
    assert max(eG, eT, eg) <= TOL and ed <= max(TOL, kappa * 1e-14)
    # the recurrent method on every entry
    rec, Tr = step(q, ctx, pr, 0)
    assert rel_err(res["G"], rec["G"]) <= TOL and rel_err(T, Tr) <= TOL
    # the step without the G output (real part of the Gram matrix only) solves the same system
    real, _ = step(q, ctx, pr, 1, want_G=False)
    assert rel_err(real["dtheta"], res["dtheta"]) <= 1e-13


@pytest.mark.parametrize("make", [lambda: W.scaled(W.config3, 14, 3, n_terms=10),
                                  lambda: W.scaled(W.config2, 13, 3, n_terms=10),
                                  lambda: W.permute_params(W.scaled(W.config5, 12, 2, n_terms=10), 8111)],
                         ids=["cfg3 n14 P84", "cfg2 n13 P78", "cfg5 n12 P72 permuted"])
def test_states_complex64(env, make):
    """complex64 storage: the kept states are FP32, the Gram matrix converts
    them exactly and forms every product in FP64; against complex128 at the
    random-walk rounding bound of the sweeps (8 sqrt(M) u, M gates).  FP32
    registers sweep four columns at a time; the lowest block then has one to
    three columns below column 1 (P = 84: top 3; P = 78: top 1; P = 72: top 3),
    whose phi registers go to the dummy state."""
    q, ctx = env
    pr = make()
    r64, T64 = step(q, ctx, pr, 1, prec="c64")
    assert ctx.stats()["block_columns"] == 4
    r128, T128 = step(q, ctx, pr, 0, prec="c128")
    bound = 8 * np.sqrt(pr.n_gates) * U32
    eG, eT = rel_err(r64["G"], r128["G"]), rel_err(T64, T128)
    say(f"{pr.name} c64 states vs c128: |dG|={eG:.2e} |dT|={eT:.2e} bound {bound:.1e}")
    assert eG <= bound and eT <= bound


def test_states_rejections(env):
    q, ctx = env
    pr = W.scaled(W.config1, 6, 2, n_terms=3)
    # the block-diagonal metric keeps to the recurrence
    ctx.set_metric_blocks([b % 2 for b in range(pr.n_params)])
    try:
        with pytest.raises(q.QNGError) as e:
            step(q, ctx, pr, 1)
        assert e.value.name == "QNG_E_UNSUPPORTED"
    finally:
        ctx.set_metric_blocks(None)
    pr = W.scaled(W.config1, 14, 2, n_terms=3)
    # the Gram matrix's partial sums alone take 8 MiB at 14 qubits
    ctx.set_mem_limit(4 << 20)
    try:
        with pytest.raises(q.QNGError) as e:
            step(q, ctx, pr, 1)
        assert e.value.name == "QNG_E_OUT_OF_MEMORY"
        with pytest.raises(q.QNGError) as e:
            ctx.set_option(q.OPT_STATE_CHUNK, -1)
        assert e.value.name == "QNG_E_INVALID_ARG"
    finally:
        ctx.set_mem_limit(0)


@pytest.mark.parametrize("make,chunk", [
    (lambda: W.controlled_circuit(7, 40, 8120, n_terms=5), 0),
    (lambda: W.controlled_layers(12, 2, 6, 8121), 0),
    (lambda: W.controlled_layers(11, 2, 6, 8122), 9),
    (lambda: W.controlled_circuit(3, 14, 8123, n_terms=3), 0)],
    ids=["random n7", "ring n12", "ring n11 chunks of 9", "random n3"])
def test_states_controlled(env, make, chunk):
    """Controlled rotations in the derivative-state variant: the no-product
    sweeps with the controlled handlers (exact plane rotations, so they add no
    sign to the kept states), columns whose top or the rotation below it is
    controlled seeded with the generator, the diagonals 1/4 Prob(control = 1)
    taken on the forward register; against the oracle, and the recurrence on
    every entry."""
    q, ctx = env
    pr = make()
    if pr.n_qubits == 7:
        pr.in_state = W.random_state(7, 8124)
    res, T, k = chunked(q, ctx, pr, chunk, "c128")
    assert k == 1 if chunk == 0 else k > 1
    want = oracle.step(pr)
    kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(pr.n_params))
    eG, eT = rel_err(res["G"], want["G"]), rel_err(T, want["T"])
    eg, ed = rel_err(res["grad"], want["grad"]), rel_err(res["dtheta"], want["dtheta"])
    say(f"{pr.name} (chunk {chunk}): |dG|={eG:.2e} |dT|={eT:.2e} |dgrad|={eg:.2e} |ddtheta|={ed:.2e}")
    assert max(eG, eT, eg) <= TOL and ed <= max(TOL, kappa * 1e-14)
    rec, Tr = step(q, ctx, pr, 0)
    assert rel_err(res["G"], rec["G"]) <= TOL and rel_err(T, Tr) <= TOL
    # complex64 against complex128 at the sweeps' rounding bound
    r64, T64, _ = chunked(q, ctx, pr, chunk, "c64")
    bound = 8 * np.sqrt(pr.n_gates) * U32
    assert rel_err(r64["G"], res["G"]) <= bound and rel_err(T64, T) <= bound


def chunked(q, ctx, pr, chunk, prec, want_G=True):
    ctx.set_option(q.OPT_STATE_CHUNK, chunk)
    try:
        res, T = step(q, ctx, pr, 1, prec=prec, want_G=want_G)
        chunks = ctx.stats()["state_chunks"]   # of the last call (the metric)
    finally:
        ctx.set_option(q.OPT_STATE_CHUNK, 0)
    return res, T, chunks


def expected_chunks(P, width, chunk):
    """Whole column blocks of `width` from the top column P - 1 down, the lowest
    block cut at column 1, grouped from the bottom into chunks of at most
    `chunk` columns."""
    blocks, top = [], P - 1
    while top >= 1:
        blocks.append(top - max(1, top - width + 1) + 1)
        top -= width
    blocks.reverse()
    if chunk == 0 or chunk >= P - 1:
        return 1
    n, cur = 0, None
    for b in blocks:
        if cur is None or cur + b > chunk:
            n, cur = n + 1, 0
        cur += b
    return n


@pytest.mark.parametrize("make,chunk,prec", [
    (lambda: W.scaled(W.config2, 13, 3, n_terms=10), 5, "c128"),
    (lambda: W.scaled(W.config3, 14, 3, n_terms=10), 10, "c64"),
    (lambda: W.permute_params(W.scaled(W.config5, 12, 2, n_terms=10), 8111), 36, "c64"),
    (lambda: W.random_circuit(3, 14, 8102, n_terms=4), 1, "c128"),
    (lambda: W.share_params(W.random_circuit(11, 60, 8106, n_terms=5), 9, 8107), 7, "c128")],
    ids=["cfg2 n13 P78 small chunks", "cfg3 n14 P84 c64 chunks of 8", "cfg5 n12 P72 c64 two chunks",
         "n3 chunks of one block", "shared n11 small chunks"])
def test_states_chunked(env, make, chunk, prec):
    """The derivative-state variant a chunk of column blocks at a time: chunk i's
    states paired with every lower chunk's (prepared again for each), against
    the oracle, against the unchunked run (every entry, to rounding: the Gram
    sums run in another order) and with the step without the G output."""
    q, ctx = env
    pr = make()
    if pr.n_qubits == 3:
        pr.in_state = W.random_state(3, 8108)
    res, T, k = chunked(q, ctx, pr, chunk, prec)
    width = ctx.stats()["block_columns"]
    assert width in (1, 2, 4) and (prec == "c128" or width == 4)
    n_rot = int((pr.gates[:, 3] >= 0).sum())   # columns: one per parameterised gate
    want_k = expected_chunks(n_rot, width, max(chunk, width))   # (a chunk holds one block at least)
    say(f"{pr.name} {prec}: chunks of <= {chunk} columns -> {k} chunks (expected {want_k})")
    assert k == want_k and k > 1
    full, Tf, k1 = chunked(q, ctx, pr, 0, prec)
    assert k1 == 1
    eG, eT = rel_err(res["G"], full["G"]), rel_err(T, Tf)
    eg = rel_err(res["grad"], full["grad"])
    say(f"{pr.name}: chunked vs unchunked |dG|={eG:.2e} |dT|={eT:.2e} |dgrad|={eg:.2e}")
    # the forward state reaches a chunk's first block through other kernels than
    # in the unchunked run (and leaves the metric phase at another gate): the
    # same up to rounding, FP32 rounding for complex64 (the sweeps' random-walk
    # bound, as for complex64 against complex128)
    tol = 1e-12 if prec == "c128" else 8 * np.sqrt(pr.n_gates) * U32
    assert eG <= tol and eT <= tol and eg <= tol
    if prec == "c128":
        want = oracle.step(pr)
        kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(pr.n_params))
        eG, eT = rel_err(res["G"], want["G"]), rel_err(T, want["T"])
        ed = rel_err(res["dtheta"], want["dtheta"])
        say(f"{pr.name}: chunked vs oracle |dG|={eG:.2e} |dT|={eT:.2e} |ddtheta|={ed:.2e}")
        assert eG <= TOL and eT <= TOL and ed <= max(TOL, kappa * 1e-14)
    # the step without the G output: the same real parts; T's imaginary parts
    # (zero but for rounding, since <y|sigma|y> is real) are then not taken
    # from the Gram matrix, which moves Re G by their products (u^2 for complex64)
    real, _, _ = chunked(q, ctx, pr, chunk, prec, want_G=False)
    kappa = np.linalg.cond(res["G"].real + pr.tikhonov * np.eye(pr.n_params))
    tol = 1e-13 if prec == "c128" else max(1e-13, kappa * (8 * np.sqrt(pr.n_gates) * U32) ** 2)
    assert rel_err(real["dtheta"], res["dtheta"]) <= tol


def test_states_chunked_by_memory(env):
    """With a memory limit under what P + 2 kept states need, the chunks are
    chosen to fit (two chunks and three more states kept at once)."""
    q, ctx = env
    pr = W.scaled(W.config1, 14, 2, n_terms=3)
    full, Tf, k1 = chunked(q, ctx, pr, 0, "c128")
    assert k1 == 1
    # 58 kept states of 256 KiB (14.5 MiB) and 8 MiB of Gram partial sums do not fit in 16 MiB
    ctx.set_mem_limit(16 << 20)
    try:
        res, T, k = chunked(q, ctx, pr, 0, "c128")
    finally:
        ctx.set_mem_limit(0)
    say(f"{pr.name}: 16 MiB limit -> {k} chunks")
    assert k > 2
    assert rel_err(res["G"], full["G"]) <= 1e-12 and rel_err(T, Tf) <= 1e-12
    want = oracle.step(pr)
    assert rel_err(res["G"], want["G"]) <= TOL


@pytest.mark.timeout(900)
def test_states_n20_full_oracle(env):
    q, ctx = env
    pr = W.config2()
    say(f"case: {pr.name} derivative-state metric, full oracle")
    res, T = step(q, ctx, pr, 1)
    D, psi = oracle.derivative_states(pr)
    Go, To, _ = oracle.metric_from_states(D, psi)
    Eo, go = oracle.energy_grad(pr, None, D=D, psi=psi)
    del D, psi
    dth = oracle.solve_step(Go, go, pr.dt, pr.tikhonov)
    kappa = np.linalg.cond(Go.real + pr.tikhonov * np.eye(pr.n_params))
    eG, eT, eg, ed = rel_err(res["G"], Go), rel_err(T, To), rel_err(res["grad"], go), rel_err(res["dtheta"], dth)
    say(f"{pr.name}: |dG|={eG:.2e} |dT|={eT:.2e} |dgrad|={eg:.2e} |ddtheta|={ed:.2e} kappa={kappa:.1e}")
    assert max(eG, eT, eg) <= TOL and ed <= max(TOL, kappa * 1e-14)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("chunk", [0, 144], ids=["all kept", "chunks of 144"])
def test_states_n24_against_recurrence(env, chunk):
    """n=24, P=432 (108 GiB of kept states; in chunks of 144 columns, 291
    states or 73 GiB): every entry against the recurrent method, which the
    full-size tests pin to the oracle."""
    q, ctx = env
    pr = W.config5()
    say(f"case: {pr.name} derivative-state metric (chunk {chunk}) vs recurrence, every entry")
    res, T, k = chunked(q, ctx, pr, chunk, "c128")
    assert k == (1 if chunk == 0 else 3)
    rec, Tr = step(q, ctx, pr, 0)
    eG, eT, eg = rel_err(res["G"], rec["G"]), rel_err(T, Tr), rel_err(res["grad"], rec["grad"])
    kappa = np.linalg.cond(rec["G"].real + pr.tikhonov * np.eye(pr.n_params))
    ed = rel_err(res["dtheta"], rec["dtheta"])
    say(f"{pr.name}: |dG|={eG:.2e} |dT|={eT:.2e} |dgrad|={eg:.2e} |ddtheta|={ed:.2e} kappa={kappa:.1e}")
    assert max(eG, eT, eg) <= TOL and ed <= max(TOL, kappa * 1e-14)
