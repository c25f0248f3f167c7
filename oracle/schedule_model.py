"""Primitive-level model of the paper's schedules, with operation counters.

TEST INFRASTRUCTURE ONLY.  The paper builds every algorithm from three
primitives -- clone a state, apply a gate (or its adjoint, derivative or
derivative-adjoint) to a state, and take an inner product (abstract; appendix
introduction).  This module runs Alg. 1 (Sec. 3) and the appendix
algorithms on small numpy state vectors through a ``Machine`` that counts each
primitive, so that tests can check (i) that each schedule produces the same
L, T and G as the definition, and (ii) the operation counts of the appendix
table of costs.

Parameterised "gates" U_k are blocks: the rotation carrying theta_k followed
by the fixed gates that come after it in the gate list (fixed gates before the
first rotation are folded into the input state).  The state only depends on
the product of all gates, so this grouping leaves psi(theta), and hence G,
unchanged.  dU_k = F_k dR_k with dR_k = (i/2) sigma_k R_k (Sec. 2,
Pauli-generator form).
"""
from __future__ import annotations

import numpy as np

_SIGMA = {
    0: np.array([[0, 1], [1, 0]], dtype=np.complex128),
    1: np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    2: np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def _apply_1q(psi: np.ndarray, n: int, q: int, m: np.ndarray) -> None:
    v = psi.reshape(2 ** (n - q - 1), 2, 2 ** q)
    a, b = v[:, 0, :].copy(), v[:, 1, :].copy()
    v[:, 0, :] = m[0, 0] * a + m[0, 1] * b
    v[:, 1, :] = m[1, 0] * a + m[1, 1] * b


def _apply_fixed(psi: np.ndarray, n: int, g, adjoint: bool) -> None:
    kind, q0, q1 = int(g[0]), int(g[1]), int(g[2])
    idx = np.arange(psi.shape[0])
    if kind == 3:   # CNOT is its own inverse
        src = idx ^ (((idx >> q0) & 1) << q1)
        psi[:] = psi[src]
    else:           # CZ is its own inverse
        psi[((idx >> q0) & 1 & (idx >> q1)) == 1] *= -1


class Circuit:
    """Blocks U_1..U_P of a gate list, in parameter (not gate-list) order is NOT
    assumed: blocks follow the gate list, and ``param[k]`` maps block k to its
    parameter index."""

    def __init__(self, problem):
        self.n = problem.n_qubits
        self.theta = problem.theta
        self.lead = []
        self.blocks = []    # (kind, qubit, param, [fixed gates after])
        for g in problem.gates:
            if int(g[3]) >= 0:
                self.blocks.append([int(g[0]), int(g[1]), int(g[3]), []])
            elif self.blocks:
                self.blocks[-1][3].append(g)
            else:
                self.lead.append(g)
        self.P = len(self.blocks)
        self.param = [b[2] for b in self.blocks]

    def rot(self, k: int, deriv: bool) -> np.ndarray:
        kind, _, p, _ = self.blocks[k]
        s = _SIGMA[kind]
        th = float(self.theta[p])
        r = np.cos(th / 2) * np.eye(2) + 1j * np.sin(th / 2) * s
        return 0.5j * s @ r if deriv else r

    def input_state(self, problem) -> np.ndarray:
        if problem.in_state is not None:
            v = np.array(problem.in_state, dtype=np.complex128)
        else:
            v = np.zeros(2 ** self.n, dtype=np.complex128)
            v[0] = 1.0
        for g in self.lead:
            _apply_fixed(v, self.n, g, False)
        return v


class Machine:
    """Counts the three primitives; registers are tracked by name."""

    def __init__(self, circ: Circuit):
        self.c = circ
        self.gates = 0
        self.clones = 0
        self.prods = 0
        self.registers = set()

    def clone(self, name: str, src: np.ndarray) -> np.ndarray:
        self.clones += 1
        self.registers.add(name)
        return src.copy()

    def apply(self, psi: np.ndarray, k: int, adjoint: bool = False, deriv: bool = False) -> None:
        """psi <- U_k, U_k^dag, dU_k or dU_k^dag (block k, 0-based)."""
        self.gates += 1
        c = self.c
        _, q, _, fixed = c.blocks[k]
        m = c.rot(k, deriv)
        if not adjoint:
            _apply_1q(psi, c.n, q, m)
            for g in fixed:
                _apply_fixed(psi, c.n, g, False)
        else:
            for g in reversed(fixed):
                _apply_fixed(psi, c.n, g, True)
            _apply_1q(psi, c.n, q, m.conj().T)

    def prod(self, a: np.ndarray, b: np.ndarray) -> complex:
        self.prods += 1
        return complex(np.vdot(a, b))


def _unpack(P: int, L: np.ndarray, T: np.ndarray, param) -> np.ndarray:
    """G_ij = L_ij - T_i^* T_j (i <= j), L_ji^* - T_i^* T_j (i > j) (Alg. 1 unpack),
    then relabelled from block order to parameter order."""
    Gb = np.empty((P, P), dtype=np.complex128)
    for i in range(P):
        for j in range(P):
            Lij = L[i, j] if i <= j else np.conj(L[j, i])
            Gb[i, j] = Lij - np.conj(T[i]) * T[j]
    G = np.empty_like(Gb)
    pi = np.asarray(param)
    G[np.ix_(pi, pi)] = Gb
    Tp = np.empty_like(T)
    Tp[pi] = T
    return G, Tp


def algorithm1(problem):
    """Alg. 1 (Sec. 3): full G with registers chi, psi, phi, lambda, mu."""
    c = Circuit(problem)
    m = Machine(c)
    P = c.P
    vin = c.input_state(problem)
    L = np.zeros((P, P), dtype=np.complex128)
    T = np.zeros(P, dtype=np.complex128)
    # edge case j = 1
    chi = m.clone("chi", vin)
    m.apply(chi, 0)
    psi = m.clone("psi", chi)
    phi = m.clone("phi", vin)
    m.apply(phi, 0, deriv=True)
    T[0] = m.prod(chi, phi)
    L[0, 0] = m.prod(phi, phi)
    for j in range(1, P):
        lam = m.clone("lambda", psi)
        phi = m.clone("phi", psi)
        m.apply(phi, j, deriv=True)
        L[j, j] = m.prod(phi, phi)
        for i in range(j - 1, -1, -1):
            m.apply(phi, i + 1, adjoint=True)
            m.apply(lam, i, adjoint=True)
            mu = m.clone("mu", lam)
            m.apply(mu, i, deriv=True)
            L[i, j] = m.prod(mu, phi)
        T[j] = m.prod(chi, phi)
        m.apply(psi, j)
    G, Tp = _unpack(P, L, T, c.param)
    return {"G": G, "T": Tp, "L_blocks": L, "counts": _counts(m)}


def _counts(m: Machine):
    return {"gates": m.gates, "clones": m.clones, "prods": m.prods, "registers": len(m.registers)}


def _L_only(problem, body):
    c = Circuit(problem)
    m = Machine(c)
    vin = c.input_state(problem)
    L = np.zeros((c.P, c.P), dtype=np.complex128)
    body(c, m, vin, L)
    return {"L_blocks": L, "counts": _counts(m), "param": c.param}


def algorithm2(problem):
    """Appendix: every element from scratch, both derivative states prepared afresh."""
    def body(c, m, vin, L):
        P = c.P
        for i in range(P):
            for j in range(P):
                a = m.clone("phiA", vin)
                b = m.clone("phiB", vin)
                for k in range(i):
                    m.apply(a, k)
                m.apply(a, i, deriv=True)
                for k in range(i + 1, P):
                    m.apply(a, k)
                for k in range(j):
                    m.apply(b, k)
                m.apply(b, j, deriv=True)
                for k in range(j + 1, P):
                    m.apply(b, k)
                L[i, j] = m.prod(a, b)
    return _L_only(problem, body)


def algorithm3(problem):
    """Appendix: i <= j only, gates after j cancelled, one register."""
    def body(c, m, vin, L):
        P = c.P
        for j in range(P):
            for i in range(j + 1):
                phi = m.clone("phi", vin)
                for k in range(j):
                    m.apply(phi, k)
                m.apply(phi, j, deriv=True)
                for k in range(j, i, -1):
                    m.apply(phi, k, adjoint=True)
                m.apply(phi, i, adjoint=True, deriv=True)
                for k in range(i - 1, -1, -1):
                    m.apply(phi, k, adjoint=True)
                L[i, j] = m.prod(vin, phi)
    return _L_only(problem, body)


def algorithm4(problem):
    """Appendix: rolling suffix state."""
    def body(c, m, vin, L):
        P = c.P
        psi = m.clone("psi", vin)
        for j in range(P):
            phi = m.clone("phi", psi)
            m.apply(phi, j, deriv=True)
            for i in range(j + 1):
                lam = m.clone("lambda", phi)
                for k in range(j, i, -1):
                    m.apply(lam, k, adjoint=True)
                m.apply(lam, i, adjoint=True, deriv=True)
                for k in range(i - 1, -1, -1):
                    m.apply(lam, k, adjoint=True)
                L[i, j] = m.prod(vin, lam)
            m.apply(psi, j)
    return _L_only(problem, body)


def algorithm5(problem):
    """Appendix: rolling suffix and infix."""
    def body(c, m, vin, L):
        P = c.P
        psi = m.clone("psi", vin)
        for j in range(P):
            phi = m.clone("phi", psi)
            m.apply(phi, j, deriv=True)
            for i in range(j, -1, -1):
                lam = m.clone("lambda", phi)
                m.apply(lam, i, adjoint=True, deriv=True)
                for k in range(i - 1, -1, -1):
                    m.apply(lam, k, adjoint=True)
                L[i, j] = m.prod(vin, lam)
                m.apply(phi, i, adjoint=True)
            m.apply(psi, j)
    return _L_only(problem, body)


def algorithm6(problem):
    """Appendix: rolling suffix, infix and prefix (Alg. 1 without T)."""
    def body(c, m, vin, L):
        P = c.P
        psi = m.clone("psi", vin)
        for j in range(P):
            mu = m.clone("mu", psi)
            phi = m.clone("phi", psi)
            m.apply(phi, j, deriv=True)
            for i in range(j, -1, -1):
                lam = m.clone("lambda", phi)
                m.apply(lam, i, adjoint=True, deriv=True)
                L[i, j] = m.prod(mu, lam)
                m.apply(phi, i, adjoint=True)
                if i > 0:
                    m.apply(mu, i - 1, adjoint=True)
            m.apply(psi, j)
    return _L_only(problem, body)


def algorithm7(problem):
    """Appendix: P independent derivative states, inner products at the end."""
    def body(c, m, vin, L):
        P = c.P
        states = []
        for i in range(P):
            s = m.clone(f"phi{i}", vin)
            for k in range(i):
                m.apply(s, k)
            m.apply(s, i, deriv=True)
            for k in range(i + 1, P):
                m.apply(s, k)
            states.append(s)
        for j in range(P):
            for i in range(j + 1):
                L[i, j] = m.prod(states[i], states[j])
    return _L_only(problem, body)


def algorithm8(problem):
    """Appendix: P derivative states from a rolling suffix (prefix) state."""
    def body(c, m, vin, L):
        P = c.P
        psi = m.clone("psi", vin)
        states = []
        for i in range(P):
            s = m.clone(f"phi{i}", psi)
            m.apply(s, i, deriv=True)
            for k in range(i + 1, P):
                m.apply(s, k)
            states.append(s)
            m.apply(psi, i)
        for j in range(P):
            for i in range(j + 1):
                L[i, j] = m.prod(states[i], states[j])
    return _L_only(problem, body)


ALGORITHMS = {1: algorithm1, 2: algorithm2, 3: algorithm3, 4: algorithm4, 5: algorithm5,
              6: algorithm6, 7: algorithm7, 8: algorithm8}


def L_in_param_order(result) -> np.ndarray:
    """Upper-triangle L (block order) -> full Hermitian L in parameter order."""
    Lb = result["L_blocks"]
    P = Lb.shape[0]
    full = np.triu(Lb) + np.triu(Lb, 1).conj().T
    param = result.get("param")
    if param is None:
        return full
    out = np.empty_like(full)
    pi = np.asarray(param)
    out[np.ix_(pi, pi)] = full
    return out


# Table of costs (appendix), as printed: (registers, gates(P), clones(P)).
TABLE1 = {
    2: (2, lambda P: 2 * P ** 3, lambda P: 2 * P ** 2),
    3: (1, lambda P: 2 * P ** 3 / 3 + P ** 2 + P / 3, lambda P: P ** 2 / 2 + P / 2),
    4: (3, lambda P: P ** 3 / 3 + P ** 2 / 2 + 13 * P / 6, lambda P: P ** 2 / 2 + 3 * P / 2 + 1),
    5: (3, lambda P: P ** 3 / 6 + P ** 2 + 11 * P / 6, lambda P: P ** 2 / 2 + 3 * P / 2 + 1),
    6: (4, lambda P: 3 * P ** 2 / 2 + 3 * P / 2, lambda P: P ** 2 / 2 + 5 * P / 2 + 1),
    7: ("P", lambda P: P ** 2 + P, lambda P: P),
    8: ("P+1", lambda P: P ** 2 / 2 + 3 * P / 2, lambda P: P + 1),
}
