"""Plain FP64 CPU oracle for the quantum natural gradient.

TEST INFRASTRUCTURE ONLY: only ``tests/``, the smoke check and the CPU-baseline
leg of ``bench.py`` may import this package.  The product library never calls
it, and it shares no code with the HIP path.

Definitions followed (Jones, "Efficient classical calculation of the Quantum
Natural Gradient"):

* ansatz state psi = U_P ... U_1 |in> (Sec. 2, problem statement);
* quantum geometric tensor G_ij = <d_i psi, d_j psi> - <d_i psi, psi><psi, d_j psi>
  (Sec. 1, definition of the geometric tensor);
* T_i = <psi, d_i psi> (Sec. 2, first definition);  L_ij = <d_i psi, d_j psi>
  (Sec. 2, definition of the Li tensor);
* energy gradient: the vector of partial derivatives of <E> = <psi|H|psi>
  (Sec. 1); for Hermitian H, d_i E = 2 Re <H psi | d_i psi>;
* natural-gradient step g dtheta = -dt grad E with g = Re G (Sec. 1), solved
  here with a Tikhonov shift: (Re G + eps I) dtheta = -dt grad E.

The derivative states come from ``oracle.c`` (gate by gate, with the entrywise
derivative of the parameterised gate's matrix); everything else is a numpy
library product or solve on those states.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    c_int, c_p = ctypes.c_int, ctypes.c_void_p
    lib.oracle_forward.argtypes = [c_int, c_int, c_p, c_p, c_p, c_p, c_p]
    lib.oracle_derivative_states.argtypes = [c_int, c_int, c_p, c_p, c_p, c_int, c_p, c_p, c_p, c_p]
    lib.oracle_apply_pauli_sum.argtypes = [c_int, c_int, c_p, c_p, c_p, c_p]
    lib.oracle_apply_pauli_letter.argtypes = [c_int, c_int, c_int, c_p]
    lib.oracle_apply_gate.argtypes = [c_int, c_p, c_p, c_int, c_p, c_p]
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _strings(strings, n):
    """The Pauli-string table of kind-8 gates as contiguous uint8 (n letters per string)."""
    if strings is None:
        return None
    return np.ascontiguousarray(np.asarray(strings, dtype=np.uint8).reshape(-1, n))


def _prep(problem):
    gates = np.ascontiguousarray(problem.gates, dtype=np.int32)
    theta = np.ascontiguousarray(problem.theta, dtype=np.float64)
    ins = None if problem.in_state is None else np.ascontiguousarray(problem.in_state, dtype=np.complex128)
    return gates, theta, ins, _strings(getattr(problem, "strings", None), problem.n_qubits)


def forward(problem) -> np.ndarray:
    """psi = U|in>, every gate in list order."""
    lib = _load()
    gates, theta, ins, strings = _prep(problem)
    out = np.empty(2 ** problem.n_qubits, dtype=np.complex128)
    lib.oracle_forward(problem.n_qubits, gates.shape[0], _ptr(gates), _ptr(theta), _ptr(ins), _ptr(out),
                       _ptr(strings))
    return out


def derivative_states(problem, sel: Optional[Sequence[int]] = None):
    """(D, psi): D[a] = d psi / d theta_{sel[a]} (rolling-prefix derivative states)."""
    lib = _load()
    gates, theta, ins, strings = _prep(problem)
    if sel is None:
        sel = range(problem.n_params)
    sel = np.ascontiguousarray(np.asarray(list(sel), dtype=np.int32))
    dim = 2 ** problem.n_qubits
    D = np.empty((sel.shape[0], dim), dtype=np.complex128)
    psi = np.empty(dim, dtype=np.complex128)
    rc = lib.oracle_derivative_states(problem.n_qubits, gates.shape[0], _ptr(gates), _ptr(theta), _ptr(ins),
                                      sel.shape[0], _ptr(sel), _ptr(D), _ptr(psi), _ptr(strings))
    if rc != 0:
        raise ValueError(f"oracle_derivative_states failed ({rc})")
    return D, psi


def metric_from_states(D: np.ndarray, psi: np.ndarray):
    """(G, T, L) from derivative states: L = <d_i|d_j>, T_i = <psi|d_i>, G = L - T_i^* T_j."""
    L = D.conj() @ D.T
    T = D @ psi.conj()
    G = L - np.outer(T.conj(), T)
    return G, T, L


def metric(problem, sel: Optional[Sequence[int]] = None):
    """(G, T) for the selected parameters (all P by default), from the definition."""
    D, psi = derivative_states(problem, sel)
    G, T, _ = metric_from_states(D, psi)
    return G, T


def apply_hamiltonian(problem, psi: np.ndarray) -> np.ndarray:
    lib = _load()
    pauli = np.ascontiguousarray(problem.pauli, dtype=np.uint8)
    coeff = np.ascontiguousarray(problem.coeff, dtype=np.float64)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    lib.oracle_apply_pauli_sum(problem.n_qubits, coeff.shape[0], _ptr(pauli), _ptr(coeff), _ptr(psi), _ptr(out))
    return out


def energy(problem) -> float:
    psi = forward(problem)
    return float(np.vdot(psi, apply_hamiltonian(problem, psi)).real)


def energy_grad(problem, sel: Optional[Sequence[int]] = None, D=None, psi=None):
    """(E, grad) with grad[a] = 2 Re <H psi | d_{sel[a]} psi>."""
    if D is None:
        D, psi = derivative_states(problem, sel)
    hpsi = apply_hamiltonian(problem, psi)
    E = float(np.vdot(psi, hpsi).real)
    grad = 2.0 * (D @ hpsi.conj()).real
    return E, grad


def solve_step(G: np.ndarray, grad: np.ndarray, dt: float, tikhonov: float) -> np.ndarray:
    """dtheta solving (Re G + eps I) dtheta = -dt grad (numpy library solve)."""
    g = G.real + tikhonov * np.eye(G.shape[0])
    return np.linalg.solve(g, -dt * grad)


def step(problem):
    """Full natural-gradient step from the definitions: dict(G, T, E, grad, dtheta)."""
    D, psi = derivative_states(problem)
    G, T, _ = metric_from_states(D, psi)
    E, grad = energy_grad(problem, D=D, psi=psi)
    dtheta = solve_step(G, grad, problem.dt, problem.tikhonov)
    return {"G": G, "T": T, "E": E, "grad": grad, "dtheta": dtheta, "psi": psi}


def apply_gate(n: int, gate, theta, psi: np.ndarray, derivative: bool = False, strings=None) -> np.ndarray:
    """One gate row applied to a copy of psi (used by convention tests)."""
    lib = _load()
    g = np.ascontiguousarray(np.asarray(gate, dtype=np.int32))
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    st = _strings(strings, n)
    lib.oracle_apply_gate(n, _ptr(g), _ptr(th), int(derivative), _ptr(out), _ptr(st))
    return out


def apply_pauli_letter(n: int, q: int, letter: int, psi: np.ndarray) -> np.ndarray:
    lib = _load()
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    lib.oracle_apply_pauli_letter(n, q, letter, _ptr(out))
    return out
