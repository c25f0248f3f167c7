"""Pins of the FP64 CPU oracle to facts fixed by the paper and by mathematics.

None of these tests retypes the oracle's own formulas: each compares it with a
closed form derived by hand from the definitions, with an independent dense
route (scipy matrix exponential + Kronecker products), with an exact identity
(parameter shift), with finite differences, or with a structural invariant.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import dense
import workloads as W


def _problem(n, gates, theta, in_state=None, pauli=None, coeff=None):
    gates = np.asarray(gates, dtype=np.int32).reshape(-1, 4)
    if pauli is None:
        pauli = np.zeros((1, n), dtype=np.uint8)
        coeff = np.zeros(1)
    return W.Problem(name="t", n_qubits=n, gates=gates, theta=np.asarray(theta, dtype=np.float64),
                     pauli=np.asarray(pauli, dtype=np.uint8), coeff=np.asarray(coeff, dtype=np.float64),
                     in_state=in_state)


# ------------------------------------------------------------------ conventions

def test_rotation_convention_matches_matrix_exponential():
    """R_sigma(theta) = exp(+i theta sigma/2) (Sec. 2 rotation example): compare
    the oracle's gate on every basis state with scipy's expm route."""
    rng = np.random.default_rng(5)
    for kind in (W.RX, W.RY, W.RZ):
        th = rng.uniform(0, 2 * np.pi, size=1)
        for q in range(3):
            for deriv in (False, True):
                u = dense.gate_unitary(3, (kind, q, -1, 0), th, derivative=deriv)
                for x in range(8):
                    e = np.zeros(8, dtype=np.complex128)
                    e[x] = 1
                    got = oracle.apply_gate(3, (kind, q, -1, 0), th, e, derivative=deriv)
                    np.testing.assert_allclose(got, u[:, x], atol=1e-15)


def test_rx_on_zero_closed_form():
    """exp(i t X/2)|0> = cos(t/2)|0> + i sin(t/2)|1> (hand expansion of the exponential)."""
    t = 0.7
    e = np.array([1, 0], dtype=np.complex128)
    got = oracle.apply_gate(1, (W.RX, 0, -1, 0), [t], e)
    np.testing.assert_allclose(got, [math.cos(t / 2), 1j * math.sin(t / 2)], atol=1e-15)


def test_fixed_gates_on_basis_states():
    """CNOT flips the target iff the control is 1; CZ negates |11>; qubit q = bit q."""
    for x in range(8):
        e = np.zeros(8, dtype=np.complex128)
        e[x] = 1
        got = oracle.apply_gate(3, (W.CNOT, 0, 2, -1), [0.0], e)
        y = x ^ (4 if x & 1 else 0)
        assert got[y] == 1 and np.count_nonzero(got) == 1
        got = oracle.apply_gate(3, (W.CZ, 1, 2, -1), [0.0], e)
        assert got[x] == (-1 if (x & 2) and (x & 4) else 1)


def test_pauli_sum_matches_dense_kronecker():
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 4):
        pr = W.random_circuit(n, 4, seed=10 + n, n_terms=5)
        pr.in_state = W.random_state(n, 20 + n)
        got = oracle.apply_hamiltonian(pr, pr.in_state)
        want = dense.hamiltonian(pr) @ pr.in_state
        np.testing.assert_allclose(got, want, atol=1e-13)
    del rng


# --------------------------------------------------------- dense brute force

@pytest.mark.parametrize("n,ngates,seed", [(1, 5, 1), (2, 9, 2), (3, 14, 3), (4, 18, 4), (4, 25, 5), (3, 30, 6)])
def test_oracle_matches_dense_brute_force(n, ngates, seed):
    pr = W.random_circuit(n, ngates, seed, n_terms=6)
    if seed % 2 == 0:
        pr.in_state = W.random_state(n, seed + 100)
    bf = dense.brute_force(pr)
    st = oracle.step(pr)
    np.testing.assert_allclose(st["psi"], bf["psi"], atol=1e-13)
    np.testing.assert_allclose(st["G"], bf["G"], atol=1e-13)
    np.testing.assert_allclose(st["T"], bf["T"], atol=1e-13)
    assert abs(st["E"] - bf["E"]) < 1e-12
    np.testing.assert_allclose(st["grad"], bf["grad"], atol=1e-12)


def test_oracle_matches_dense_on_small_hea():
    pr = W.scaled(W.config1, 4, 2, n_terms=8)
    bf = dense.brute_force(pr)
    st = oracle.step(pr)
    np.testing.assert_allclose(st["G"], bf["G"], atol=1e-13)
    np.testing.assert_allclose(st["grad"], bf["grad"], atol=1e-12)
    pr = W.scaled(W.config5, 3, 2, n_terms=8)
    bf = dense.brute_force(pr)
    st = oracle.step(pr)
    np.testing.assert_allclose(st["G"], bf["G"], atol=1e-13)
    np.testing.assert_allclose(st["grad"], bf["grad"], atol=1e-12)


# ------------------------------------------------------------- closed forms
# Single layers on |0...0> with no entanglers give product states, so G is
# block diagonal over qubits.  Per qubit (paper's +i convention):
#   RY(a): psi = (c, -s), d_a psi = (-s/2, -c/2)          -> G_aa = 1/4, T_a = 0
#   RY(a) then RZ(b): psi = (c e^{ib/2}, -s e^{-ib/2})
#       d_b psi = (i/2)(c e^{ib/2}, s e^{-ib/2})          -> T_b = (i/2) cos a,
#       G_bb = 1/4 - |T_b|^2 = sin^2(a)/4,  G_ab = <d_a|d_b> = -(i/4) sin a
#   RX(a) then RY(b): T_a = 0, T_b = (i/2) sin a, G_bb = cos^2(a)/4,
#       G_ab = (1/4)<phi|XY|phi> = (i/4) cos a,  phi = RX(a)|0> = (c, i s)
# (c = cos(a/2), s = sin(a/2)).

def test_closed_form_ry_layer_and_rx_layer():
    n = 5
    rng = np.random.default_rng(7)
    for kind in (W.RY, W.RX):
        gates = [(kind, q, -1, q) for q in range(n)]
        pr = _problem(n, gates, rng.uniform(0, 2 * np.pi, n))
        G, T = oracle.metric(pr)
        np.testing.assert_allclose(G, 0.25 * np.eye(n), atol=1e-15)
        np.testing.assert_allclose(T, 0, atol=1e-15)


def test_closed_form_ry_then_rz():
    n = 4
    rng = np.random.default_rng(8)
    a = rng.uniform(0, 2 * np.pi, n)
    b = rng.uniform(0, 2 * np.pi, n)
    gates = [(W.RY, q, -1, q) for q in range(n)] + [(W.RZ, q, -1, n + q) for q in range(n)]
    pr = _problem(n, gates, np.concatenate([a, b]))
    G, T = oracle.metric(pr)
    want = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    for q in range(n):
        want[q, q] = 0.25
        want[n + q, n + q] = 0.25 * math.sin(a[q]) ** 2
        want[q, n + q] = -0.25j * math.sin(a[q])
        want[n + q, q] = 0.25j * math.sin(a[q])
    np.testing.assert_allclose(G, want, atol=1e-15)
    np.testing.assert_allclose(T[n:], 0.5j * np.cos(a), atol=1e-15)
    np.testing.assert_allclose(T[:n], 0, atol=1e-15)


def test_closed_form_rx_then_ry():
    n = 3
    rng = np.random.default_rng(9)
    a = rng.uniform(0, 2 * np.pi, n)
    b = rng.uniform(0, 2 * np.pi, n)
    gates = [(W.RX, q, -1, q) for q in range(n)] + [(W.RY, q, -1, n + q) for q in range(n)]
    pr = _problem(n, gates, np.concatenate([a, b]))
    G, T = oracle.metric(pr)
    want = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    for q in range(n):
        want[q, q] = 0.25
        want[n + q, n + q] = 0.25 * math.cos(a[q]) ** 2
        want[q, n + q] = 0.25j * math.cos(a[q])
        want[n + q, q] = -0.25j * math.cos(a[q])
    np.testing.assert_allclose(G, want, atol=1e-15)
    np.testing.assert_allclose(T[n:], 0.5j * np.sin(a), atol=1e-15)


def test_leading_rz_on_zero_state_has_zero_row():
    """RZ first on |0>: only the global phase moves, so its G row and column vanish;
    G_jj = 1/4 - |T_j|^2 with |T_j| = 1/2."""
    pr = W.scaled(W.config3, 4, 1)
    gates = np.concatenate([[[W.RZ, 2, -1, pr.n_params]], pr.gates]).astype(np.int32)
    pr2 = _problem(4, gates, np.concatenate([pr.theta, [1.234]]))
    G, T = oracle.metric(pr2)
    p = pr.n_params
    np.testing.assert_allclose(G[p, :], 0, atol=1e-15)
    np.testing.assert_allclose(G[:, p], 0, atol=1e-15)
    assert abs(abs(T[p]) - 0.5) < 1e-15


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("cfg,n,layers", [(W.config1, 6, 3), (W.config2, 5, 3), (W.config5, 5, 2), (W.config3, 7, 2)])
def test_metric_invariants(cfg, n, layers):
    pr = W.scaled(cfg, n, layers)
    G, T = oracle.metric(pr)
    np.testing.assert_allclose(G, G.conj().T, atol=1e-14)            # Hermitian
    assert np.linalg.eigvalsh(G).min() > -1e-12                       # PSD
    assert np.linalg.eigvalsh(G.real).min() > -1e-12                  # Re G PSD
    np.testing.assert_allclose(T.real, 0, atol=1e-14)                 # <psi|psi>=1 => Re T = 0
    assert np.abs(T).max() <= 0.5 + 1e-14
    np.testing.assert_allclose(np.diag(G).real, 0.25 - np.abs(T) ** 2, atol=1e-14)  # L_ii = 1/4
    np.testing.assert_allclose(np.diag(G).imag, 0, atol=1e-14)


def test_trailing_fixed_gates_leave_G_unchanged():
    pr = W.scaled(W.config1, 5, 2)
    G0, T0 = oracle.metric(pr)
    extra = np.array([[W.CNOT, 0, 3, -1], [W.CZ, 1, 4, -1], [W.CNOT, 4, 2, -1]], dtype=np.int32)
    pr2 = _problem(5, np.concatenate([pr.gates, extra]), pr.theta)
    G1, T1 = oracle.metric(pr2)
    np.testing.assert_allclose(G1, G0, atol=1e-14)


def test_two_pi_shift_and_global_phase_invariance():
    pr = W.scaled(W.config5, 4, 2, n_terms=6)
    pr.in_state = W.random_state(4, 77)
    st0 = oracle.step(pr)
    th = pr.theta.copy()
    th[[1, 5, 9]] += 2 * np.pi
    pr2 = W.Problem(**{**pr.__dict__, "theta": th})
    st1 = oracle.step(pr2)
    np.testing.assert_allclose(st1["G"], st0["G"], atol=1e-13)
    assert abs(st1["E"] - st0["E"]) < 1e-13
    pr3 = W.Problem(**{**pr.__dict__, "in_state": pr.in_state * np.exp(0.83j)})
    st3 = oracle.step(pr3)
    np.testing.assert_allclose(st3["G"], st0["G"], atol=1e-13)
    np.testing.assert_allclose(st3["grad"], st0["grad"], atol=1e-13)
    assert abs(st3["E"] - st0["E"]) < 1e-13


def test_zero_angles_z_hamiltonian_energy():
    """theta = 0 on |0..0> leaves the state |0..0> (up to CNOTs acting trivially),
    so a Z-only Hamiltonian has E = sum of coefficients."""
    pr = W.scaled(W.config3, 5, 2, n_terms=7)
    pr.theta[:] = 0.0
    pr.pauli[:] = np.where(pr.pauli == 0, 0, 3)
    assert abs(oracle.energy(pr) - pr.coeff.sum()) < 1e-14


# -------------------------------------------------------------- gradient pins

@pytest.mark.parametrize("cfg,n,layers", [(W.config1, 5, 2), (W.config2, 4, 3), (W.config5, 4, 2)])
def test_gradient_parameter_shift_exact(cfg, n, layers):
    """For single-Pauli rotations dE/dtheta_p = [E(theta + pi/2 e_p) - E(theta - pi/2 e_p)]/2."""
    pr = W.scaled(cfg, n, layers, n_terms=9)
    E, grad = oracle.energy_grad(pr)
    shift = np.empty_like(grad)
    for p in range(pr.n_params):
        vals = []
        for s in (+1, -1):
            th = pr.theta.copy()
            th[p] += s * np.pi / 2
            vals.append(oracle.energy(W.Problem(**{**pr.__dict__, "theta": th})))
        shift[p] = 0.5 * (vals[0] - vals[1])
    np.testing.assert_allclose(grad, shift, atol=1e-12)


def test_gradient_central_finite_difference():
    pr = W.scaled(W.config3, 4, 2, n_terms=6)
    E, grad = oracle.energy_grad(pr)
    h = 1e-6
    fd = np.empty_like(grad)
    for p in range(pr.n_params):
        th = pr.theta.copy(); th[p] += h
        ep = oracle.energy(W.Problem(**{**pr.__dict__, "theta": th}))
        th[p] -= 2 * h
        em = oracle.energy(W.Problem(**{**pr.__dict__, "theta": th}))
        fd[p] = (ep - em) / (2 * h)
    np.testing.assert_allclose(grad, fd, atol=1e-8 * max(1.0, abs(E)))


def test_metric_is_fubini_study_second_order():
    """Re G is the Fubini-Study metric: 1 - |<psi(t)|psi(t+d)>|^2 = d^T (Re G) d + O(|d|^3)."""
    pr = W.scaled(W.config2, 4, 2)
    G, _ = oracle.metric(pr)
    psi0 = oracle.forward(pr)
    rng = np.random.default_rng(11)
    d = rng.standard_normal(pr.n_params)
    d /= np.linalg.norm(d)
    for eps in (1e-3, 5e-4):
        psi1 = oracle.forward(W.Problem(**{**pr.__dict__, "theta": pr.theta + eps * d}))
        lhs = 1 - abs(np.vdot(psi0, psi1)) ** 2
        rhs = eps ** 2 * d @ G.real @ d
        assert abs(lhs - rhs) < 5 * eps ** 3


# ------------------------------------------------------------------ the step

def test_step_on_flat_metric_is_scaled_gradient():
    """RY layer on |0..0>: G = I/4, so dtheta = -dt grad / (1/4 + eps) exactly."""
    n = 5
    pr = W.make_problem("ry", n, 1, (W.RY,), "none", 6, seed=3)
    st = oracle.step(pr)
    np.testing.assert_allclose(st["dtheta"], -pr.dt * st["grad"] / (0.25 + pr.tikhonov), rtol=1e-13, atol=1e-16)


def test_step_descends_and_predicts_energy_change():
    pr = W.scaled(W.config1, 5, 2, n_terms=10)
    pr.dt = 1e-3
    st = oracle.step(pr)
    assert st["grad"] @ st["dtheta"] < 0
    E1 = oracle.energy(W.Problem(**{**pr.__dict__, "theta": pr.theta + st["dtheta"]}))
    lin = st["grad"] @ st["dtheta"]
    assert abs((E1 - st["E"]) - lin) < 50 * np.linalg.norm(st["dtheta"]) ** 2 * (1 + np.abs(pr.coeff).sum())


# ---------------------------------------------------- sampled entries route

def test_selected_entries_match_full_metric():
    """The column-subset route (derivative states for a few parameters) gives the
    same entries as the full P x P evaluation."""
    pr = W.scaled(W.config3, 6, 2)
    G, T = oracle.metric(pr)
    sel = [0, 5, 6, 11, 17, pr.n_params - 1]
    Gs, Ts = oracle.metric(pr, sel)
    np.testing.assert_allclose(Gs, G[np.ix_(sel, sel)], atol=1e-15)
    np.testing.assert_allclose(Ts, T[sel], atol=1e-15)


def test_parameter_relabelling_permutes_outputs():
    pr = W.scaled(W.config5, 4, 1)
    pp = W.permute_params(pr, 5)
    G, T = oracle.metric(pr)
    Gp, Tp = oracle.metric(pp)
    rng = np.random.default_rng(5)
    perm = rng.permutation(pr.n_params)
    np.testing.assert_allclose(Gp[np.ix_(perm, perm)], G, atol=1e-15)
    np.testing.assert_allclose(Tp[perm], T, atol=1e-15)


# ------------------------------------------------------- shared parameters

def test_shared_parameter_derivatives_match_finite_differences():
    """A parameter carried by several gates: d psi / d theta_a (the sum of the
    gates' terms) against central differences of the forward state, whose
    error is h^2/6 |psi'''| <= h^2/6 (k/2)^3 for k gates carrying the angle."""
    pr = W.share_params(W.random_circuit(5, 40, 901, n_terms=5), 6, 902)
    D, psi = oracle.derivative_states(pr)
    h = 1e-5
    for a in range(pr.n_params):
        k = int((pr.gates[:, 3] == a).sum())
        assert k >= 1
        tp, tm = pr.theta.copy(), pr.theta.copy()
        tp[a] += h
        tm[a] -= h
        fd = (oracle.forward(W.Problem(**{**pr.__dict__, "theta": tp}))
              - oracle.forward(W.Problem(**{**pr.__dict__, "theta": tm}))) / (2 * h)
        assert np.abs(D[a] - fd).max() < h * h / 6 * (k / 2) ** 3 + 1e-9


def test_shared_rx_pair_closed_form():
    """RX(theta) twice on one qubit, one shared angle: the state is RX(2 theta)|0>,
    so d psi/d theta is twice the single-gate derivative at 2 theta and
    G = 4 * 1/4 = 1, T = 2 * (i/2) <psi|X|psi> = 0 (|<X>| = 0 on RX|0>)."""
    g = np.array([[W.RX, 0, -1, 0], [W.RX, 0, -1, 0]], dtype=np.int32)
    pr = W.Problem("rx_pair", 1, g, np.array([0.7]), np.array([[3]], np.uint8), np.array([1.0]))
    G, T = oracle.metric(pr)
    np.testing.assert_allclose(G, [[1.0]], atol=1e-15)
    np.testing.assert_allclose(T, [0.0], atol=1e-15)
    # energy <Z> = cos(2 theta): gradient -2 sin(2 theta)
    E, grad = oracle.energy_grad(pr)
    np.testing.assert_allclose([E, grad[0]], [math.cos(1.4), -2 * math.sin(1.4)], atol=1e-14)


def test_shared_parameters_contract_the_unshared_metric():
    """Relabelling merges parameters: G' = J^T G J and grad' = J^T grad, where
    G, grad belong to the same circuit with one parameter per gate (J maps
    each gate's parameter to the shared one).  Checks the oracle's sum of
    derivative terms against its one-gate-per-parameter evaluation."""
    base = W.random_circuit(5, 36, 903, n_terms=5)
    pr = W.share_params(base, 5, 904)
    unshared = W.Problem(**{**base.__dict__, "theta": pr.theta[pr.gates[pr.gates[:, 3] >= 0, 3]][
        np.argsort(base.gates[base.gates[:, 3] >= 0, 3])]})
    J = np.zeros((base.n_params, pr.n_params))
    J[base.gates[base.gates[:, 3] >= 0, 3], pr.gates[pr.gates[:, 3] >= 0, 3]] = 1.0
    G, _ = oracle.metric(unshared)
    Gs, _ = oracle.metric(pr)
    np.testing.assert_allclose(Gs, J.T @ G @ J, atol=1e-13)
    _, g = oracle.energy_grad(unshared)
    _, gs = oracle.energy_grad(pr)
    np.testing.assert_allclose(gs, J.T @ g, atol=1e-13)


def test_dense_route_sums_derivative_terms_of_a_shared_parameter():
    """The dense brute force with shared angles: d U / d theta_a is the sum over
    the gates carrying a (product rule), checked against central differences of
    the dense unitary itself (error h^2/6 times the third derivative, at most
    (k/2)^3 for k gates carrying the angle), and its G and gradient against the
    oracle's C route on the same problem."""
    pr = W.share_params(W.random_circuit(3, 16, 905, n_terms=4), 3, 906)
    assert any(int((pr.gates[:, 3] == a).sum()) > 1 for a in range(pr.n_params))
    h = 1e-5
    for a in range(pr.n_params):
        k = int((pr.gates[:, 3] == a).sum())
        tp, tm = pr.theta.copy(), pr.theta.copy()
        tp[a] += h
        tm[a] -= h
        fd = (dense.unitary(W.Problem(**{**pr.__dict__, "theta": tp}))
              - dense.unitary(W.Problem(**{**pr.__dict__, "theta": tm}))) / (2 * h)
        assert np.abs(dense.derivative_unitary(pr, a) - fd).max() < h * h / 6 * (k / 2) ** 3 + 1e-9
    bf = dense.brute_force(pr)
    st = oracle.step(pr)
    np.testing.assert_allclose(st["G"], bf["G"], atol=1e-13)
    np.testing.assert_allclose(st["grad"], bf["grad"], atol=1e-12)


# ------------------------------------------------------ controlled rotations

def test_controlled_rotation_on_basis_states():
    """A controlled rotation leaves every basis state whose control bit is 0
    untouched and rotates the target of the others (the gate of Sec. 2's
    controlled-rotation example); its derivative vanishes where the control
    is 0.  Checked against the plain rotation applied to a 1-qubit target."""
    rng = np.random.default_rng(41)
    for kind, plain in ((W.CRX, W.RX), (W.CRY, W.RY), (W.CRZ, W.RZ)):
        th = rng.uniform(0, 2 * np.pi, size=1)
        for deriv in (False, True):
            r = np.stack([oracle.apply_gate(1, (plain, 0, -1, 0), th, e, derivative=deriv)
                          for e in np.eye(2, dtype=np.complex128)], axis=1)
            for x in range(8):
                e = np.zeros(8, dtype=np.complex128)
                e[x] = 1
                got = oracle.apply_gate(3, (kind, 2, 0, 0), th, e, derivative=deriv)
                want = np.zeros(8, dtype=np.complex128)
                if x & 4:
                    t = x & 1
                    want[x & ~1] = r[0, t]
                    want[x | 1] = r[1, t]
                elif not deriv:
                    want[x] = 1
                np.testing.assert_allclose(got, want, atol=1e-15)
                u = dense.gate_unitary(3, (kind, 2, 0, 0), th, derivative=deriv)
                np.testing.assert_allclose(got, u[:, x], atol=1e-15)


def test_controlled_closed_forms():
    """Control prepared as cos(a)|0> + sin(a)|1> (p = sin^2 a), target |0>.
    CRY(theta): psi = cos a |00> + sin a |1> RY|0>, and RY(theta)|0> is real, so
    <Y> = 0 there: T = 0 and G = p/4.  CRZ(theta): RZ|0> is an eigenvector of
    Z with eigenvalue 1, so <psi|d psi> = i p/2 and G = p/4 - p^2/4."""
    for a in (0.3, math.pi / 4, 1.2):
        p = math.sin(a) ** 2
        ins = np.zeros(4, dtype=np.complex128)
        ins[0], ins[1] = math.cos(a), math.sin(a)           # qubit 0 = control, qubit 1 = target
        for kind, G_want, T_want in ((W.CRY, p / 4, 0.0), (W.CRZ, p / 4 - p * p / 4, 0.5j * p)):
            pr = _problem(2, [[kind, 0, 1, 0]], [0.9], in_state=ins)
            G, T = oracle.metric(pr)
            np.testing.assert_allclose(G, [[G_want]], atol=1e-15)
            np.testing.assert_allclose(T, [T_want], atol=1e-15)


def test_controlled_diagonal_is_quarter_control_probability():
    """Sec. 2: for a controlled rotation L_ii = 1/4 <psi_{i-1}| (|1><1| on the
    control) |psi_{i-1}>, with psi_{i-1} the state just before gate i; for a
    plain rotation L_ii = 1/4."""
    pr = W.controlled_circuit(5, 40, 411, n_terms=4)
    pr.in_state = W.random_state(5, 412)
    D, psi = oracle.derivative_states(pr)
    L = np.einsum("ix,ix->i", D.conj(), D).real
    state = pr.in_state.copy()
    for g in pr.gates:
        kind, q0, _, p = (int(v) for v in g)
        if p >= 0:
            if kind >= W.CRX:
                idx = np.arange(1 << pr.n_qubits)
                prob = float(np.sum(np.abs(state[(idx >> q0) & 1 == 1]) ** 2))
                assert abs(L[p] - prob / 4) < 1e-14
            else:
                assert abs(L[p] - 0.25) < 1e-14
        state = oracle.apply_gate(pr.n_qubits, g, pr.theta, state)


@pytest.mark.parametrize("n,ngates,seed", [(2, 12, 421), (3, 20, 422), (4, 30, 423), (5, 26, 424)])
def test_controlled_oracle_matches_dense_brute_force(n, ngates, seed):
    pr = W.controlled_circuit(n, ngates, seed, n_terms=6)
    if seed % 2 == 0:
        pr.in_state = W.random_state(n, seed + 100)
    bf = dense.brute_force(pr)
    st = oracle.step(pr)
    np.testing.assert_allclose(st["psi"], bf["psi"], atol=1e-13)
    np.testing.assert_allclose(st["G"], bf["G"], atol=1e-13)
    np.testing.assert_allclose(st["T"], bf["T"], atol=1e-13)
    assert abs(st["E"] - bf["E"]) < 1e-12
    np.testing.assert_allclose(st["grad"], bf["grad"], atol=1e-12)


def test_controlled_derivatives_match_finite_differences():
    """d psi / d theta of controlled rotations (alone and with a shared angle)
    against central differences of the forward state; error <= h^2/6 (k/2)^3."""
    base = W.controlled_circuit(4, 30, 431, n_terms=4)
    for pr in (base, W.share_params(base, 5, 432)):
        D, _ = oracle.derivative_states(pr)
        h = 1e-5
        for a in range(pr.n_params):
            k = int((pr.gates[:, 3] == a).sum())
            tp, tm = pr.theta.copy(), pr.theta.copy()
            tp[a] += h
            tm[a] -= h
            fd = (oracle.forward(W.Problem(**{**pr.__dict__, "theta": tp}))
                  - oracle.forward(W.Problem(**{**pr.__dict__, "theta": tm}))) / (2 * h)
            assert np.abs(D[a] - fd).max() < h * h / 6 * (k / 2) ** 3 + 1e-9


def test_controlled_gradient_four_term_shift():
    """A controlled rotation's generator |1><1| (x) sigma/2 has eigenvalues
    0, +-1/2, so E(theta) is a trigonometric polynomial of frequencies 1/2 and
    1; the four-term shift rule with shifts pi/2 and 3pi/2 (coefficients
    (sqrt2 + 1)/(4 sqrt2) and (sqrt2 - 1)/(4 sqrt2)) gives the exact derivative."""
    pr = W.controlled_layers(3, 2, 7, 441)
    E, grad = oracle.energy_grad(pr)
    c1 = (math.sqrt(2) + 1) / (4 * math.sqrt(2))
    c2 = (math.sqrt(2) - 1) / (4 * math.sqrt(2))
    for p in range(pr.n_params):
        def e(shift):
            th = pr.theta.copy()
            th[p] += shift
            return oracle.energy(W.Problem(**{**pr.__dict__, "theta": th}))
        d = c1 * (e(math.pi / 2) - e(-math.pi / 2)) - c2 * (e(3 * math.pi / 2) - e(-3 * math.pi / 2))
        assert abs(d - grad[p]) < 1e-12, (p, d, grad[p])


# ------------------------------------------------ the element-by-element route

@pytest.mark.parametrize("make", [lambda: W.random_circuit(3, 11, 451, n_terms=3),
                                  lambda: W.controlled_circuit(3, 9, 452, n_terms=3)])
def test_each_element_prepared_independently(make):
    """Alg. 2 of the appendix (each element from two states, each prepared from
    |in> on its own, P <= 8), with dense gate matrices: every
    L_ij = <phi_A|phi_B>, where phi_A is the ansatz with gate i replaced by its
    derivative and phi_B the same for j; T_i = <psi|phi_A>; G = L - T^* T."""
    pr = make()
    pr.in_state = W.random_state(pr.n_qubits, 453)
    P, n = pr.n_params, pr.n_qubits
    assert 2 <= P <= 8

    def prepare(deriv):
        v = pr.in_state.copy()
        for g in pr.gates:
            v = dense.gate_unitary(n, g, pr.theta, derivative=int(g[3]) == deriv and deriv >= 0) @ v
        return v

    psi = prepare(-1)
    L = np.empty((P, P), dtype=np.complex128)
    T = np.empty(P, dtype=np.complex128)
    for i in range(P):
        for j in range(P):
            L[i, j] = np.vdot(prepare(i), prepare(j))
        T[i] = np.vdot(psi, prepare(i))
    G, To = oracle.metric(pr)
    np.testing.assert_allclose(To, T, atol=1e-14)
    np.testing.assert_allclose(G, L - np.outer(T.conj(), T), atol=1e-14)


# ------------------------------------------------------ Pauli-string rotations

def test_string_rotation_on_basis_states():
    """exp(i t S/2) for multi-qubit strings (identity letters included) against
    scipy's matrix exponential of the dense string, and its derivative
    (i/2) S exp(i t S/2), on every basis state."""
    rng = np.random.default_rng(61)
    table = np.array([[1, 0, 3], [2, 2, 0], [3, 1, 2], [0, 0, 0], [3, 3, 3]], dtype=np.uint8)
    for k in range(table.shape[0]):
        th = rng.uniform(0, 2 * np.pi, size=1)
        for deriv in (False, True):
            u = dense.gate_unitary(3, (W.RPAULI, k, -1, 0), th, derivative=deriv, strings=table)
            for x in range(8):
                e = np.zeros(8, dtype=np.complex128)
                e[x] = 1
                got = oracle.apply_gate(3, (W.RPAULI, k, -1, 0), th, e, derivative=deriv, strings=table)
                np.testing.assert_allclose(got, u[:, x], atol=1e-15)


def test_single_letter_string_is_the_plain_rotation():
    rng = np.random.default_rng(62)
    psi = W.random_state(3, 63)
    for letter, kind in ((1, W.RX), (2, W.RY), (3, W.RZ)):
        for q in range(3):
            table = np.zeros((1, 3), dtype=np.uint8)
            table[0, q] = letter
            th = rng.uniform(0, 2 * np.pi, size=1)
            for deriv in (False, True):
                a = oracle.apply_gate(3, (W.RPAULI, 0, -1, 0), th, psi, derivative=deriv, strings=table)
                b = oracle.apply_gate(3, (kind, q, -1, 0), th, psi, derivative=deriv)
                np.testing.assert_allclose(a, b, atol=1e-15)


def test_string_closed_forms():
    """ZZ rotation on cos a|x=0> + sin a|x=2> (ZZ eigenvalues +1, -1): <S> =
    cos 2a, so T = (i/2) cos 2a and G = (1 - cos^2 2a)/4; the X^{(x)3} rotation
    on |000>: psi = cos(t/2)|000> + i sin(t/2)|111>, so with H = Z_0,
    E = cos t and dE/dt = -sin t."""
    table = np.array([[3, 3]], dtype=np.uint8)
    for a in (0.2, 0.7, 1.3):
        ins = np.zeros(4, dtype=np.complex128)
        ins[0], ins[2] = math.cos(a), math.sin(a)
        pr = _problem(2, [[W.RPAULI, 0, -1, 0]], [1.1], in_state=ins)
        pr.strings = table
        G, T = oracle.metric(pr)
        np.testing.assert_allclose(G, [[(1 - math.cos(2 * a) ** 2) / 4]], atol=1e-15)
        np.testing.assert_allclose(T, [0.5j * math.cos(2 * a)], atol=1e-15)
    for t in (0.4, 2.5):
        pr = _problem(3, [[W.RPAULI, 0, -1, 0]], [t], pauli=[[3, 0, 0]], coeff=[1.0])
        pr.strings = np.array([[1, 1, 1]], dtype=np.uint8)
        E, g = oracle.energy_grad(pr)
        np.testing.assert_allclose([E, g[0]], [math.cos(t), -math.sin(t)], atol=1e-14)


@pytest.mark.parametrize("n,ngates,seed", [(2, 10, 461), (3, 18, 462), (4, 26, 463), (4, 16, 464)])
def test_string_oracle_matches_dense_brute_force(n, ngates, seed):
    pr = W.string_circuit(n, ngates, seed, n_terms=6)
    if seed % 2 == 0:
        pr.in_state = W.random_state(n, seed + 100)
    bf = dense.brute_force(pr)
    st = oracle.step(pr)
    np.testing.assert_allclose(st["psi"], bf["psi"], atol=1e-13)
    np.testing.assert_allclose(st["G"], bf["G"], atol=1e-13)
    np.testing.assert_allclose(st["T"], bf["T"], atol=1e-13)
    assert abs(st["E"] - bf["E"]) < 1e-12
    np.testing.assert_allclose(st["grad"], bf["grad"], atol=1e-12)


def test_string_gradient_two_term_shift_and_derivatives():
    """A Pauli string has eigenvalues +-1, so the two-term shift rule is exact
    for its angle; derivative states against central differences."""
    pr = W.string_layers(4, 2, 7, 471)
    E, grad = oracle.energy_grad(pr)
    for p in range(pr.n_params):
        vals = []
        for s_ in (+1, -1):
            th = pr.theta.copy()
            th[p] += s_ * np.pi / 2
            vals.append(oracle.energy(W.Problem(**{**pr.__dict__, "theta": th})))
        assert abs(0.5 * (vals[0] - vals[1]) - grad[p]) < 1e-12
    D, _ = oracle.derivative_states(pr)
    h = 1e-5
    for a in range(pr.n_params):
        tp, tm = pr.theta.copy(), pr.theta.copy()
        tp[a] += h
        tm[a] -= h
        fd = (oracle.forward(W.Problem(**{**pr.__dict__, "theta": tp}))
              - oracle.forward(W.Problem(**{**pr.__dict__, "theta": tm}))) / (2 * h)
        assert np.abs(D[a] - fd).max() < h * h / 6 / 8 + 1e-9
