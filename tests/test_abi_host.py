"""CPU-only checks of the C ABI library: it loads, exports every symbol the
header declares, and its host-only logic (validation, error codes, solve) is
correct.  No compute entry point is called without a GPU."""
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qng.h")


@pytest.fixture(scope="module")
def qng():
    import paper_2011_02991_amd as q
    return q


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:qng_status|void|const char \*)\s*(qng_\w+)\s*\(", text, re.M)))


def test_header_symbols_exported(qng):
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(qng.lib(), s), s
    assert sorted(qng.EXPORTED) == syms


def _circ(qng, pr):
    return qng.Circuit.from_problem(pr)


def test_validate_accepts_workloads(qng):
    for cfg in (W.config1, W.config2, W.config3, W.config5):
        pr = cfg()
        qng.validate(_circ(qng, pr), pr.theta)
    for pr in W.config4()[:5]:
        qng.validate(_circ(qng, pr), pr.theta)


@pytest.mark.parametrize("mutate,status", [
    (lambda g: g.__setitem__((0, 1), 99), "QNG_E_BAD_CIRCUIT"),          # qubit out of range
    (lambda g: g.__setitem__((0, 0), 11), "QNG_E_BAD_CIRCUIT"),          # unknown kind
    (lambda g: g.__setitem__((1, 3), 0), "QNG_E_BAD_PARAMS"),            # parameter 1 left on no rotation
    (lambda g: g.__setitem__((0, 2), 3), "QNG_E_BAD_CIRCUIT"),           # rotation with q1 != -1
])
def test_validate_rejects_bad_circuits(qng, mutate, status):
    pr = W.scaled(W.config1, 4, 1)
    g = pr.gates.copy()
    mutate(g)
    with pytest.raises(qng.QNGError) as e:
        qng.validate(qng.Circuit(4, g, pr.n_params, pr.pauli, pr.coeff), pr.theta)
    assert e.value.name == status


def test_validate_accepts_shared_parameters(qng):
    """Several rotations may carry one parameter (n_params < rotations)."""
    pr = W.layer_shared(5, 3, 6, 11)
    assert pr.n_params == 6 and int((pr.gates[:, 3] >= 0).sum()) == 30
    qng.validate(_circ(qng, pr), pr.theta)
    pr2 = W.share_params(W.random_circuit(6, 30, 12), 4, 13)
    qng.validate(_circ(qng, pr2), pr2.theta)


def test_validate_controlled_rotations(qng):
    """CRX/CRY/CRZ (kinds 5/6/7): control q0, target q1, a parameter index."""
    for pr in (W.controlled_circuit(6, 40, 21), W.controlled_layers(5, 2, 4, 22)):
        assert (pr.gates[:, 0] >= W.CRX).any()
        qng.validate(_circ(qng, pr), pr.theta)
    bad = [([W.CRY, 1, 1, 0], "QNG_E_BAD_CIRCUIT"),     # control == target
           ([W.CRX, 0, 5, 0], "QNG_E_BAD_CIRCUIT"),     # target out of range
           ([W.CRZ, -1, 1, 0], "QNG_E_BAD_CIRCUIT"),    # control out of range
           ([W.CRZ, 0, 1, -1], "QNG_E_BAD_PARAMS"),     # no parameter
           ([W.CRZ, 0, 1, 2], "QNG_E_BAD_PARAMS")]      # parameter >= n_params
    for row, status in bad:
        g = np.array([[W.RY, 0, -1, 0], row], dtype=np.int32)
        with pytest.raises(qng.QNGError) as e:
            qng.validate(qng.Circuit(2, g, 1), [0.1], with_hamiltonian=False)
        assert e.value.name == status, (row, e.value.name)


def test_validate_pauli_string_rotations(qng):
    """RPAULI (kind 8): q0 indexes the circuit's string table, q1 = -1."""
    for pr in (W.string_circuit(6, 40, 31), W.string_layers(5, 2, 4, 32)):
        assert (pr.gates[:, 0] == W.RPAULI).any()
        qng.validate(_circ(qng, pr), pr.theta)
    table = np.array([[1, 3], [0, 2]], dtype=np.uint8)
    bad = [([W.RPAULI, 2, -1, 0], table, "QNG_E_BAD_CIRCUIT"),     # string index out of range
           ([W.RPAULI, -1, -1, 0], table, "QNG_E_BAD_CIRCUIT"),
           ([W.RPAULI, 0, 1, 0], table, "QNG_E_BAD_CIRCUIT"),      # q1 != -1
           ([W.RPAULI, 0, -1, -1], table, "QNG_E_BAD_PARAMS"),     # no parameter
           ([W.RPAULI, 1, -1, 0], np.array([[1, 3], [0, 4]], np.uint8), "QNG_E_BAD_CIRCUIT")]   # letter 4
    for row, tab, status in bad:
        g = np.array([[W.RY, 0, -1, 0], row], dtype=np.int32)
        with pytest.raises(qng.QNGError) as e:
            qng.validate(qng.Circuit(2, g, 1, strings=tab), [0.1], with_hamiltonian=False)
        assert e.value.name == status, (row, e.value.name)
    c = qng.Circuit(2, np.array([[W.RPAULI, 0, -1, 0]], np.int32), 1, strings=table)
    c.c.strings = None
    with pytest.raises(qng.QNGError) as e:
        qng.validate(c, [0.1], with_hamiltonian=False)
    assert e.value.name == "QNG_E_INVALID_ARG"


def test_fused_planner_takes_controlled_rotations_and_strings(qng):
    """Controlled rotations are planned onto the fused passes (every element
    once), and so are Pauli-string rotations, rewritten as basis rotations,
    CNOTs and an RZ (more gates, the same elements); the export of a plan with
    strings (whose rows would name positions of the rewritten list) and the
    fused plan of a string without letters are rejected (QNG_E_UNSUPPORTED)."""
    pr = W.controlled_layers(6, 2, 4, 23)
    c = _circ(qng, pr)
    P = pr.n_params
    for fusion in (0, 1):
        assert qng.plan(c, fusion=fusion)["elements"] == P * (P - 1) // 2
    assert qng.plan(c, fusion=1)["passes"] > 0
    assert len(qng.plan_export(c)) > 0
    pr = W.string_layers(6, 2, 4, 24)
    c = _circ(qng, pr)
    P = pr.n_params
    for fusion in (0, 1):
        assert qng.plan(c, fusion=fusion)["elements"] == P * (P - 1) // 2
    assert qng.plan(c, fusion=1)["passes"] > 0
    with pytest.raises(qng.QNGError) as e:
        qng.plan_export(c)
    assert e.value.name == "QNG_E_UNSUPPORTED"
    table = np.zeros((1, 3), dtype=np.uint8)
    g = np.array([[W.RY, 0, -1, 0], [W.RPAULI, 0, -1, 1], [W.RY, 1, -1, 2]], dtype=np.int32)
    c = qng.Circuit(3, g, 3, strings=table)
    assert qng.plan(c, fusion=0)["elements"] == 3
    with pytest.raises(qng.QNGError) as e:
        qng.plan(c, fusion=1)
    assert e.value.name == "QNG_E_UNSUPPORTED"


def test_validate_two_qubit_gate_same_qubit(qng):
    g = np.array([[W.RY, 0, -1, 0], [W.CNOT, 1, 1, -1]], dtype=np.int32)
    with pytest.raises(qng.QNGError) as e:
        qng.validate(qng.Circuit(2, g, 1), [0.1], with_hamiltonian=False)
    assert e.value.name == "QNG_E_BAD_CIRCUIT"


def test_validate_missing_parameter(qng):
    g = np.array([[W.RY, 0, -1, 0], [W.RZ, 1, -1, 2]], dtype=np.int32)
    with pytest.raises(qng.QNGError) as e:
        qng.validate(qng.Circuit(2, g, 2), [0.1, 0.2], with_hamiltonian=False)
    assert e.value.name == "QNG_E_BAD_PARAMS"


def test_validate_nonfinite(qng):
    pr = W.scaled(W.config1, 3, 1)
    th = pr.theta.copy()
    th[2] = np.nan
    with pytest.raises(qng.QNGError) as e:
        qng.validate(_circ(qng, pr), th)
    assert e.value.name == "QNG_E_NONFINITE"
    c = qng.Circuit(3, pr.gates, pr.n_params, pr.pauli, np.where(np.arange(pr.n_terms) == 1, np.inf, pr.coeff))
    with pytest.raises(qng.QNGError) as e:
        qng.validate(c, pr.theta)
    assert e.value.name == "QNG_E_NONFINITE"


def test_validate_bad_pauli_letter(qng):
    pr = W.scaled(W.config1, 3, 1)
    p = pr.pauli.copy()
    p[0, 0] = 4
    with pytest.raises(qng.QNGError) as e:
        qng.validate(qng.Circuit(3, pr.gates, pr.n_params, p, pr.coeff), pr.theta)
    assert e.value.name == "QNG_E_INVALID_ARG"


def test_solve_shifted_matches_numpy(qng):
    rng = np.random.default_rng(1)
    P = 37
    A = rng.standard_normal((P, P)) + 1j * rng.standard_normal((P, P))
    G = A @ A.conj().T / P
    b = rng.standard_normal(P)
    x = qng.solve_shifted(G, 1e-4, b)
    want = np.linalg.solve(G.real + 1e-4 * np.eye(P), b)
    np.testing.assert_allclose(x, want, rtol=1e-10, atol=1e-12)


def test_solve_shifted_not_spd(qng):
    G = np.zeros((3, 3), dtype=np.complex128)
    G[0, 0] = 1.0
    with pytest.raises(qng.QNGError) as e:
        qng.solve_shifted(G, 0.0, np.ones(3))
    assert e.value.name == "QNG_E_NOT_SPD"


def test_create_without_gpu_fails_cleanly(qng):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(qng.QNGError) as e:
        qng.Context(0)
    assert e.value.name == "QNG_E_DEVICE"


def test_header_constants_match_binding(qng):
    """Option codes, status codes and the stats struct of the header agree with
    the Python binding's marshalling."""
    text = open(HEADER).read()
    opts = dict((k, int(v)) for k, v in re.findall(r"QNG_OPT_(\w+)\s*=\s*(\d+)", text))
    for name, val in opts.items():
        assert getattr(qng, "OPT_" + name) == val, name
    status = dict((k, int(v)) for k, v in re.findall(r"(QNG_(?:OK|E_\w+))\s*=\s*(-?\d+)", text))
    for name, val in status.items():
        assert qng.STATUS[val] == name
    end = text.index("} qng_stats;")
    body = text[text.rindex("typedef struct {", 0, end):end]
    fields = re.findall(r"^\s*(int64_t|int32_t|double)\s+(\w+);", body, re.M)
    ct = {"int64_t": "c_long", "int32_t": "c_int", "double": "c_double"}
    assert [(n, ct[t]) for t, n in fields] == [(n, t.__name__) for n, t in qng.Stats._fields_]
