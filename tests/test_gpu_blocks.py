"""Blocks of two and of four metric columns sharing one lambda sweep
(QNG_OPT_BLOCK_COLUMNS = 2 or 4) against the FP64 CPU oracle.

Columns s and s - 1 (s - 3 .. s) are swept together: lambda is swept once,
phi of each lower column is seeded inside the sweep as sigma lambda where
lambda reaches its y (with <lambda|phi> there giving its T).  Four-column
blocks run in tiles of 11 qubits with FP32 registers (complex64 storage).  complex128 results must match the
oracle as in the single-column tests (1e-10 normwise); complex64 results are
checked against the same bound as the single-column complex64 path and
against the single-column complex64 result.  The workloads have registers of
11 to 16 qubits (tiles of 11 or 12 qubits, so passes mix register, thread and
tile-base locations and Z products outside the tile), even and odd P (the
lowest block then has one real column), RX/RY/RZ seeds, CNOT chains and CZ
rings, input states and permuted parameters.
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
def qng():
    import torch  # noqa: F401
    import paper_2011_02991_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(qng):
    c = qng.Context(0)
    yield c
    c.close()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300))


def step(ctx, qng, pr, prec, block, tile=0, f64=0, exact=0):
    ctx.set_option(qng.OPT_BLOCK_COLUMNS, block)
    ctx.set_option(qng.OPT_TILE_QUBITS, tile)
    ctx.set_option(qng.OPT_F64_REGISTERS, f64)
    ctx.set_option(qng.OPT_EXACT_PRODUCTS, exact)
    try:
        return ctx.step(qng.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state, prec=prec)
    finally:
        ctx.set_option(qng.OPT_BLOCK_COLUMNS, 0)
        ctx.set_option(qng.OPT_TILE_QUBITS, 0)
        ctx.set_option(qng.OPT_F64_REGISTERS, 0)
        ctx.set_option(qng.OPT_EXACT_PRODUCTS, 1)


def check(res, want, pr, label):
    eG, eT = rel_err(res["G"], want["G"]), 0.0
    eg = rel_err(res["grad"], want["grad"])
    ed = rel_err(res["dtheta"], want["dtheta"])
    kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(pr.n_params))
    say(f"{label}: |dG|={eG:.2e} |dgrad|={eg:.2e} |ddtheta|={ed:.2e} kappa={kappa:.1e}")
    assert eG <= TOL and eg <= TOL, (eG, eg)
    assert ed <= max(TOL, kappa * 1e-14), ed


def with_state(pr, seed):
    # a random input state: from |0..0> this circuit and Hamiltonian give
    # E = 0 and a zero gradient (no relative error to check against)
    pr.in_state = W.random_state(pr.n_qubits, seed)
    return pr


CASES = [
    ("cfg3 n=12 L=2", lambda: W.scaled(W.config3, 12, 2, n_terms=9), 0),
    ("cfg2 n=13 L=2", lambda: W.scaled(W.config2, 13, 2, n_terms=9), 11),
    ("cfg5 n=14 L=2", lambda: W.scaled(W.config5, 14, 2, n_terms=9), 12),
    ("cfg1 n=15 L=1", lambda: W.scaled(W.config1, 15, 1, n_terms=9), 11),
    ("random n=13", lambda: with_state(W.random_circuit(13, 61, 4101, n_terms=6), 4104), 11),
    ("random n=12 odd P", lambda: W.random_circuit(12, 45, 4102, n_terms=6, fixed_fraction=0.3), 0),
    ("random n=16 permuted", lambda: W.permute_params(W.random_circuit(16, 40, 4103, n_terms=5), 3), 12),
]


@pytest.mark.parametrize("label,make,tile", CASES, ids=[c[0] for c in CASES])
def test_blocks_complex128(ctx, qng, label, make, tile):
    pr = make()
    say(f"case: {label} (n={pr.n_qubits}, P={pr.n_params}, tile={tile}) c128 block=2")
    res = step(ctx, qng, pr, "c128", 2, tile)
    check(res, oracle.step(pr), pr, label)


@pytest.mark.parametrize("mode", ["fp32", "fp64_registers", "exact_products"])
@pytest.mark.parametrize("label,make,tile", CASES[:5], ids=[c[0] for c in CASES[:5]])
def test_blocks_complex64(ctx, qng, label, make, tile, mode):
    """complex64 storage in each register mode: FP32 registers with FP32
    thread shares of the products (default), FP64 registers, and FP32
    registers with every product in FP64."""
    pr = make()
    f64, exact = int(mode == "fp64_registers"), int(mode == "exact_products")
    say(f"case: {label} (n={pr.n_qubits}, P={pr.n_params}) c64 {mode} block=2")
    two = step(ctx, qng, pr, "c64", 2, 0, f64, exact)
    one = step(ctx, qng, pr, "c64", 1, 0, f64, exact)
    want = oracle.step(pr)
    bound = 4 * pr.gates.shape[0] * 2.0 ** -24
    for key in ("G", "grad"):
        e2, e1 = rel_err(two[key], want[key]), rel_err(one[key], want[key])
        say(f"  {key}: block=2 {e2:.2e}, block=1 {e1:.2e} (bound {bound:.1e})")
        assert e2 <= bound and e1 <= bound
        # the two schedules round differently, within the same bound
        assert rel_err(two[key], one[key]) <= bound


def test_blocks_full_step_cfg3_n20(ctx, qng):
    """n=20 (8 qubits outside a 12-qubit tile), 2 layers, complex128 and complex64."""
    pr = W.scaled(W.config3, 20, 2, n_terms=20)
    say(f"case: cfg3 n=20 L=2 P={pr.n_params} block=2")
    want = oracle.step(pr)
    check(step(ctx, qng, pr, "c128", 2), want, pr, "cfg3 n=20 c128")
    r64 = step(ctx, qng, pr, "c64", 2)
    bound = 4 * pr.gates.shape[0] * 2.0 ** -24
    assert rel_err(r64["G"], want["G"]) <= bound and rel_err(r64["grad"], want["grad"]) <= bound


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("label,make", [("cfg3 n=14 L=2", lambda: W.scaled(W.config3, 14, 2, n_terms=9)),
                                        ("cfg5 n=13 L=2", lambda: W.scaled(W.config5, 13, 2, n_terms=9)),
                                        ("cfg2 n=9 L=3", lambda: W.scaled(W.config2, 9, 3, n_terms=9))])
def test_step_without_G_output(ctx, qng, label, make, prec):
    """Without a G output the step needs Re G only, and the fused passes keep the
    real parts of the metric's inner products (half the multiply-adds).  The
    real parts are formed by the same chains in the same order, so the step is
    the same to the last bit or close to it; against the oracle as usual."""
    pr = make()
    pr.in_state = W.random_state(pr.n_qubits, 731)
    circ = qng.Circuit.from_problem(pr)
    full = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state, prec=prec, want_G=True)
    real = ctx.step(circ, pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state, prec=prec, want_G=False)
    st = ctx.stats()
    assert st["sweep_launches"] > 0
    ed = rel_err(real["dtheta"], full["dtheta"])
    say(f"{label} {prec}: |ddtheta| real vs full {ed:.2e}")
    assert ed <= 1e-13
    assert np.array_equal(real["grad"], full["grad"]) and real["E"] == full["E"]
    want = oracle.step(pr)
    kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(pr.n_params))
    bound = TOL if prec == "c128" else 4 * pr.gates.shape[0] * 2.0 ** -24
    assert rel_err(real["dtheta"], want["dtheta"]) <= max(bound, kappa * bound if prec == "c64" else kappa * 1e-14)


FOUR = [
    ("cfg3 n=12 L=2", lambda: with_state(W.scaled(W.config3, 12, 2, n_terms=9), 4201)),
    ("cfg2 n=13 L=3", lambda: W.scaled(W.config2, 13, 3, n_terms=9)),
    ("cfg5 n=11 L=2", lambda: W.scaled(W.config5, 11, 2, n_terms=9)),
    ("random n=14 permuted P%4=3", lambda: with_state(W.permute_params(W.random_circuit(14, 80, 4202, n_terms=6), 5), 4203)),
    ("random n=15 P%4=3", lambda: with_state(W.random_circuit(15, 61, 4204, n_terms=6, fixed_fraction=0.2), 4206)),
]


@pytest.mark.parametrize("exact", [1, 0])
@pytest.mark.parametrize("label,make", FOUR, ids=[c[0] for c in FOUR])
def test_four_column_blocks_complex64(ctx, qng, label, make, exact):
    """Four columns per sweep (tiles of 11 qubits, FP32 registers): against the
    oracle at the complex64 bound and against two columns per sweep (the same
    bound: both round the stored states the same number of times), with the
    complex G (complex products) and the step without it (real parts)."""
    pr = make()
    say(f"case: {label} (n={pr.n_qubits}, P={pr.n_params}, P % 4 = {pr.n_params % 4}) c64 exact={exact} block=4")
    four = step(ctx, qng, pr, "c64", 4, 0, 0, exact)
    assert ctx.stats()["block_columns"] == 4
    two = step(ctx, qng, pr, "c64", 2, 0, 0, exact)
    want = oracle.step(pr)
    bound = 4 * pr.gates.shape[0] * 2.0 ** -24
    for key in ("G", "grad"):
        e4, e2 = rel_err(four[key], want[key]), rel_err(two[key], want[key])
        say(f"  {key}: block=4 {e4:.2e}, block=2 {e2:.2e} (bound {bound:.1e})")
        assert e4 <= bound and rel_err(four[key], two[key]) <= bound
    ctx.set_option(qng.OPT_BLOCK_COLUMNS, 4)
    ctx.set_option(qng.OPT_EXACT_PRODUCTS, exact)
    try:
        real = ctx.step(qng.Circuit.from_problem(pr), pr.theta, pr.dt, pr.tikhonov, in_state=pr.in_state,
                        prec="c64", want_G=False)
    finally:
        ctx.set_option(qng.OPT_BLOCK_COLUMNS, 0)
        ctx.set_option(qng.OPT_EXACT_PRODUCTS, 1)
    kappa = np.linalg.cond(want["G"].real + pr.tikhonov * np.eye(pr.n_params))
    ed = rel_err(real["dtheta"], four["dtheta"])
    say(f"  step without G vs with G (block=4): |ddtheta|={ed:.2e} kappa={kappa:.1e}")
    assert ed <= max(bound, kappa * bound)


def test_four_column_blocks_not_taken(ctx, qng):
    """Four columns per sweep only where they apply: complex128 and FP64
    registers, tiles other than 11 qubits, registers below 11 qubits and
    circuits with controlled rotations fall back to two columns (or one)."""
    pr = W.scaled(W.config3, 12, 1, n_terms=4)
    for prec, f64, tile in (("c128", 0, 0), ("c64", 1, 0), ("c64", 0, 12)):
        step(ctx, qng, pr, prec, 4, tile, f64, 1)
        assert ctx.stats()["block_columns"] == 2, (prec, f64, tile)
    step(ctx, qng, W.scaled(W.config3, 10, 1, n_terms=4), "c64", 4, 0, 0, 1)
    assert ctx.stats()["block_columns"] != 4
    step(ctx, qng, W.controlled_layers(12, 1, 4, 4205), "c64", 4, 0, 0, 1)
    assert ctx.stats()["block_columns"] == 2
