"""The paper's schedules run on a primitive-level model with counters.

Checks that Alg. 1 (Sec. 3) and the appendix algorithms compute the same L, T
and G as the definition-based oracle, and that their primitive counts match the
appendix table of costs and the worked totals printed in the appendix.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import schedule_model as SM
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appendix_counts.txt")


def _only_rotations(n, P, seed):
    """P parameterised rotations (no fixed gates), so that 'gates' in the counts
    are exactly the paper's parameterised gates."""
    rng = np.random.default_rng(seed)
    gates = [(int(rng.integers(0, 3)), int(rng.integers(0, n)), -1, p) for p in range(P)]
    return W.Problem(name="rot", n_qubits=n, gates=np.asarray(gates, dtype=np.int32),
                     theta=rng.uniform(0, 2 * np.pi, P), pauli=np.zeros((1, n), np.uint8),
                     coeff=np.zeros(1))


@pytest.mark.parametrize("seed", range(6))
def test_algorithm1_matches_definition(seed):
    pr = W.random_circuit(3, 12, seed=seed)
    if seed % 2:
        pr.in_state = W.random_state(3, seed)
    got = SM.algorithm1(pr)
    G, T = oracle.metric(pr)
    np.testing.assert_allclose(got["G"], G, atol=1e-13)
    np.testing.assert_allclose(got["T"], T, atol=1e-13)


def test_algorithm1_on_permuted_parameters():
    pr = W.permute_params(W.scaled(W.config1, 3, 2), 3)
    got = SM.algorithm1(pr)
    G, T = oracle.metric(pr)
    np.testing.assert_allclose(got["G"], G, atol=1e-13)


@pytest.mark.parametrize("alg", [2, 3, 4, 5, 6, 7, 8])
def test_appendix_algorithms_agree_on_L(alg):
    pr = W.random_circuit(3, 10, seed=40 + alg)
    D, psi = oracle.derivative_states(pr)
    _, _, L = oracle.metric_from_states(D, psi)
    res = SM.ALGORITHMS[alg](pr)
    np.testing.assert_allclose(SM.L_in_param_order(res), L, atol=1e-13)


@pytest.mark.parametrize("P", [1, 2, 3, 5, 8])
def test_algorithm1_counts(P):
    """Counting the primitives of Alg. 1: gates 3P^2/2 + P/2, clones P^2/2 + 3P/2 + 1,
    inner products P^2/2 + 3P/2, five registers."""
    res = SM.algorithm1(_only_rotations(2, P, P))
    c = res["counts"]
    assert c["gates"] == (3 * P * P + P) // 2
    assert c["clones"] == (P * P + 3 * P) // 2 + 1
    assert c["prods"] == (P * P + 3 * P) // 2
    assert c["registers"] == 5 if P > 1 else c["registers"] == 3


@pytest.mark.parametrize("alg", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("P", [1, 2, 4, 7])
def test_appendix_table_counts(alg, P):
    """Literal counts against the appendix table.  Algs. 5 and 6 apply one more
    gate per column than the table (the final phi <- U_1^dag of each column is
    never used); Alg. 7's table entry counts P more gates than its listing."""
    res = SM.ALGORITHMS[alg](_only_rotations(2, P, 100 + P))
    c = res["counts"]
    regs, gates_f, clones_f = SM.TABLE1[alg]
    offset = {5: P, 6: P, 7: -P}.get(alg, 0)
    assert c["gates"] == round(gates_f(P)) + offset
    assert c["clones"] == round(clones_f(P))
    if alg == 2:
        assert c["prods"] == P * P
    else:
        assert c["prods"] == (P * P + P) // 2
    want_regs = {"P": P, "P+1": P + 1}.get(regs, regs)
    assert c["registers"] == want_regs


def test_worked_totals_from_golden_file():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for alg, P, total in rows:
        alg, P, total = int(alg), int(P), int(total)
        _, gates_f, clones_f = SM.TABLE1[alg]
        assert round(gates_f(P) + clones_f(P)) == total


def test_forty_parameters_claim_arithmetic():
    """Introduction: a study with ~40 parameters could reach ~250 in the same time.
    The element-by-element algorithm at P=40 costs what the O(P^2) algorithm costs
    near P = 255 (appendix table)."""
    cost2 = lambda P: 2 * P ** 3 + 2 * P ** 2
    cost6 = lambda P: 2 * P ** 2 + 4 * P + 1
    assert cost6(254) < cost2(40) < cost6(256)
