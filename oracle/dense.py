"""Dense brute force for tiny registers (n <= 4): a second, independent route.

TEST INFRASTRUCTURE ONLY.  Every gate is tensored up to a full 2^n x 2^n
matrix with Kronecker products and the ansatz unitary is formed by matrix
products -- the O(2^{3n}) route the paper's appendix introduction rules out for
real sizes, which makes it a good independent check at n <= 4.

* rotation: scipy's matrix exponential of +i theta sigma / 2 (the paper's
  convention, Sec. 2 rotation example);
* its derivative: (i/2) sigma R(theta) (Sec. 2, Pauli-generator form); the
  derivative of U by a parameter is the product-rule sum over the gates that
  carry it (one term for a unique parameter, Sec. 2; several when shared);
* CNOT and CZ: permutation / diagonal matrices written from their action on
  basis states;
* controlled rotations (kinds 5/6/7, control q0, target q1): |0><0| (x) I +
  |1><1| (x) R on (control, target); derivative |1><1| (x) (i/2) sigma R;
* Pauli-string rotations (kind 8, string q0 of the problem's table): scipy's
  matrix exponential of +i theta S / 2 for the dense string S; derivative
  (i/2) S R;
* G, T from the definition (Sec. 1), E = <psi|H|psi>, grad E by its
  definition as a vector of partial derivatives of <E> (Sec. 1).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

_PAULI = {
    0: np.eye(2, dtype=np.complex128),
    1: np.array([[0, 1], [1, 0]], dtype=np.complex128),
    2: np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    3: np.array([[1, 0], [0, -1]], dtype=np.complex128),
}
_KIND_TO_LETTER = {0: 1, 1: 2, 2: 3, 5: 1, 6: 2, 7: 3}
_P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
_P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def embed_1q(n: int, q: int, m: np.ndarray) -> np.ndarray:
    """m acting on qubit q (bit q of the index; qubit n-1 is the leftmost factor)."""
    out = np.ones((1, 1), dtype=np.complex128)
    for k in reversed(range(n)):
        out = np.kron(out, m if k == q else np.eye(2, dtype=np.complex128))
    return out


def gate_unitary(n: int, gate, theta, derivative: bool = False, strings=None) -> np.ndarray:
    kind, q0, q1, p = (int(v) for v in gate)
    dim = 2 ** n
    if kind == 8:   # Pauli-string rotation
        s = pauli_string(n, np.asarray(strings).reshape(-1, n)[q0])
        r = scipy.linalg.expm(0.5j * float(theta[p]) * s)
        return 0.5j * s @ r if derivative else r
    if kind == 3:   # CNOT control q0 target q1
        m = np.zeros((dim, dim), dtype=np.complex128)
        for x in range(dim):
            y = x ^ ((1 << q1) if (x >> q0) & 1 else 0)
            m[y, x] = 1.0
        return m
    if kind == 4:   # CZ
        return np.diag([(-1.0) ** (((x >> q0) & 1) * ((x >> q1) & 1)) for x in range(dim)]).astype(np.complex128)
    sigma = _PAULI[_KIND_TO_LETTER[kind]]
    r = scipy.linalg.expm(0.5j * float(theta[p]) * sigma)
    if derivative:
        r = 0.5j * sigma @ r
    if kind >= 5:   # controlled rotation: control q0, target q1
        on = embed_1q(n, q0, _P1) @ embed_1q(n, q1, r)
        return on if derivative else embed_1q(n, q0, _P0) + on
    return embed_1q(n, q0, r)


def pauli_string(n: int, letters) -> np.ndarray:
    out = np.ones((1, 1), dtype=np.complex128)
    for k in reversed(range(n)):
        out = np.kron(out, _PAULI[int(letters[k])])
    return out


def hamiltonian(problem) -> np.ndarray:
    n = problem.n_qubits
    h = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    for t in range(problem.n_terms):
        h += problem.coeff[t] * pauli_string(n, problem.pauli[t])
    return h


def _input(problem) -> np.ndarray:
    if problem.in_state is not None:
        return np.asarray(problem.in_state, dtype=np.complex128)
    v = np.zeros(2 ** problem.n_qubits, dtype=np.complex128)
    v[0] = 1.0
    return v


def unitary(problem) -> np.ndarray:
    """U = G_M ... G_1, every gate in list order."""
    n = problem.n_qubits
    u = np.eye(2 ** n, dtype=np.complex128)
    for g in problem.gates:
        u = gate_unitary(n, g, problem.theta, strings=getattr(problem, "strings", None)) @ u
    return u


def derivative_unitary(problem, p: int) -> np.ndarray:
    """dU/dtheta_p by the product rule: one term per gate that carries p, that
    gate replaced by its derivative and every other gate kept (a parameter
    shared by several gates gives a sum of such terms)."""
    n = problem.n_qubits
    strings = getattr(problem, "strings", None)
    total = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    for k, gk in enumerate(problem.gates):
        if int(gk[3]) != p:
            continue
        u = np.eye(2 ** n, dtype=np.complex128)
        for j, g in enumerate(problem.gates):
            u = gate_unitary(n, g, problem.theta, derivative=(j == k), strings=strings) @ u
        total += u
    return total


def brute_force(problem):
    """dict(psi, G, T, E, grad) by dense linear algebra."""
    vin = _input(problem)
    psi = unitary(problem) @ vin
    P = problem.n_params
    D = np.stack([derivative_unitary(problem, p) @ vin for p in range(P)]) if P else np.zeros((0, psi.shape[0]))
    L = D.conj() @ D.T
    T = D @ psi.conj()
    G = L - np.outer(T.conj(), T)
    H = hamiltonian(problem)
    E = float(np.vdot(psi, H @ psi).real)
    # d<psi|H|psi>/d theta_p = <d_p psi|H|psi> + <psi|H|d_p psi>
    grad = np.array([(np.vdot(D[p], H @ psi) + np.vdot(psi, H @ D[p])).real for p in range(P)])
    return {"psi": psi, "G": G, "T": T, "L": L, "E": E, "grad": grad}
