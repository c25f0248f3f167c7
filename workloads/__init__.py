"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only *describes* problems: gate lists, angles, Pauli-sum
Hamiltonians and input states.  It applies no gate, evaluates no inner
product and holds none of the method's arithmetic, so that the oracle
(``oracle/``) and the GPU library (``paper_2011_02991_amd``) can both consume
the same inputs while sharing no code.

Problem statement (Jones, "Efficient classical calculation of the Quantum
Natural Gradient", Sec. 2, problem statement of the ansatz): an ansatz is a
product of P gates, each with its own parameter, acting on a fixed input state.
The workloads below are "hardware-efficient" layered ansaetze: each layer is a
set of single-qubit rotation sweeps followed by a fixed entangler.  Fixed
entangling gates carry parameter index -1.

Gate encoding (one row per gate, int32): ``(kind, q0, q1, param)``

* kind 0/1/2 = RX/RY/RZ on qubit q0 (q1 = -1), rotation exp(+i theta sigma/2)
  as written in Sec. 2 of the paper;
* kind 3 = CNOT with control q0 and target q1;
* kind 4 = CZ on qubits q0, q1;
* kind 5/6/7 = controlled RX/RY/RZ with control q0 and target q1 (the rotation
  acts on the target where the control is 1; Sec. 2, controlled rotations);
* kind 8 = Pauli-string rotation exp(+i theta S/2), S = the tensor product of
  the letters ``strings[q0]`` (one letter per qubit, 0..3 = I, X, Y, Z), q1 = -1.

Qubit q is bit q of the amplitude index (qubit 0 is the least significant bit).
Pauli letters are 0=I, 1=X, 2=Y, 3=Z, stored row-major as ``pauli[t, q]``.

Draw order for every seeded problem, from ``numpy.random.Generator(PCG64(seed))``:
angles (P values, uniform [0, 2 pi)), then Pauli letters (terms x n, uniform in
{0,1,2,3}), then coefficients (terms values, standard normal).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

RX, RY, RZ, CNOT, CZ = 0, 1, 2, 3, 4
CRX, CRY, CRZ = 5, 6, 7                 # controlled rotations: control q0, target q1
RPAULI = 8                              # Pauli-string rotation: q0 = row of Problem.strings
KIND_NAMES = {RX: "RX", RY: "RY", RZ: "RZ", CNOT: "CNOT", CZ: "CZ", CRX: "CRX", CRY: "CRY", CRZ: "CRZ",
              RPAULI: "RPAULI"}
ROTATION_KINDS = (RX, RY, RZ)


@dataclasses.dataclass
class Problem:
    """One QNG problem instance: circuit, angles, Hamiltonian, input state."""

    name: str
    n_qubits: int
    gates: np.ndarray            # (n_gates, 4) int32: kind, q0, q1, param
    theta: np.ndarray            # (P,) float64
    pauli: np.ndarray            # (terms, n) uint8 in {0,1,2,3}
    coeff: np.ndarray            # (terms,) float64
    in_state: Optional[np.ndarray] = None   # (2^n,) complex128, None = |0...0>
    dt: float = 0.1
    tikhonov: float = 1e-4
    seed: int = 0
    strings: Optional[np.ndarray] = None    # (k, n) uint8: letters of the kind-8 gates' Pauli strings

    @property
    def n_params(self) -> int:
        return int(self.theta.shape[0])

    @property
    def n_gates(self) -> int:
        return int(self.gates.shape[0])

    @property
    def n_terms(self) -> int:
        return int(self.coeff.shape[0])


def hea_gates(n: int, layers: int, rotations: Sequence[int], entangler: str) -> np.ndarray:
    """Gate list of a layered hardware-efficient ansatz.

    Each layer: for each rotation kind r in ``rotations``, r on every qubit
    0..n-1 in increasing order; then the entangler.  ``entangler`` is
    ``"cnot_chain"`` (CNOT q -> q+1 for q = 0..n-2, in that order),
    ``"cz_ring"`` (CZ(q, (q+1) mod n) for q = 0..n-1) or ``"none"``.
    Parameter indices follow the order in which rotations appear.
    """
    rows: List[List[int]] = []
    p = 0
    for _ in range(layers):
        for r in rotations:
            for q in range(n):
                rows.append([int(r), q, -1, p])
                p += 1
        if entangler == "cnot_chain":
            for q in range(n - 1):
                rows.append([CNOT, q, q + 1, -1])
        elif entangler == "cz_ring":
            if n == 2:
                rows.append([CZ, 0, 1, -1])
            elif n > 2:
                for q in range(n):
                    rows.append([CZ, q, (q + 1) % n, -1])
        elif entangler != "none":
            raise ValueError(f"unknown entangler {entangler!r}")
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


def draw_problem_data(seed: int, n_params: int, n_qubits: int, n_terms: int):
    """Angles, Pauli letters and coefficients in the documented draw order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.uniform(0.0, 2.0 * math.pi, size=n_params)
    pauli = rng.integers(0, 4, size=(n_terms, n_qubits)).astype(np.uint8)
    coeff = rng.standard_normal(n_terms)
    return theta.astype(np.float64), pauli, coeff.astype(np.float64)


def make_problem(name: str, n: int, layers: int, rotations: Sequence[int], entangler: str,
                 n_terms: int, seed: int, dt: float = 0.1, tikhonov: float = 1e-4) -> Problem:
    gates = hea_gates(n, layers, rotations, entangler)
    n_params = int((gates[:, 3] >= 0).sum())
    theta, pauli, coeff = draw_problem_data(seed, n_params, n, n_terms)
    return Problem(name=name, n_qubits=n, gates=gates, theta=theta, pauli=pauli,
                   coeff=coeff, dt=dt, tikhonov=tikhonov, seed=seed)


# ----------------------------------------------------------------------------
# The five workloads.  Sizes follow the synthetic hardware-efficient ansaetze
# used to exercise the method; the paper itself runs no experiments.
# ----------------------------------------------------------------------------

def config1() -> Problem:
    """n=10, 4 layers x [RY all, RZ all, CNOT chain], P=80, 20 terms."""
    return make_problem("cfg1_n10_P80", 10, 4, (RY, RZ), "cnot_chain", 20, 1001)


def config2() -> Problem:
    """n=20, 10 layers x [RX all, RY all, CZ ring], P=400, 50 terms."""
    return make_problem("cfg2_n20_P400", 20, 10, (RX, RY), "cz_ring", 50, 1002)


def config3() -> Problem:
    """n=26, 8 layers x [RY all, RZ all, CNOT chain], P=416, 100 terms."""
    return make_problem("cfg3_n26_P416", 26, 8, (RY, RZ), "cnot_chain", 100, 1003)


def config4() -> List[Problem]:
    """64 ansaetze: n_b ~ U{12..22}, L_b ~ U{2..8}, [RY, RZ, CNOT chain], 30 terms.

    The (n_b, L_b) pairs come from seed 1004 (all 64 qubit counts, then all 64
    depths); ansatz b draws its angles and Hamiltonian from seed 40000 + b.
    """
    rng = np.random.Generator(np.random.PCG64(1004))
    ns = rng.integers(12, 23, size=64)
    ls = rng.integers(2, 9, size=64)
    return [make_problem(f"cfg4_b{b}_n{int(ns[b])}_L{int(ls[b])}", int(ns[b]), int(ls[b]),
                         (RY, RZ), "cnot_chain", 30, 40000 + b) for b in range(64)]


def config5() -> Problem:
    """n=24, 6 layers x [RX all, RY all, RZ all, CZ ring], P=432, 80 terms, dt=0.05."""
    return make_problem("cfg5_n24_P432", 24, 6, (RX, RY, RZ), "cz_ring", 80, 1005, dt=0.05)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def scaled(problem_fn, n: int, layers: int, n_terms: Optional[int] = None, seed: Optional[int] = None) -> Problem:
    """A smaller instance with the same layer recipe as a named workload."""
    base = {config1: ((RY, RZ), "cnot_chain", 20, 1001),
            config2: ((RX, RY), "cz_ring", 50, 1002),
            config3: ((RY, RZ), "cnot_chain", 100, 1003),
            config5: ((RX, RY, RZ), "cz_ring", 80, 1005)}[problem_fn]
    rots, ent, terms, s = base
    return make_problem(f"{problem_fn.__name__}_scaled_n{n}_L{layers}", n, layers, rots, ent,
                        n_terms if n_terms is not None else terms,
                        seed if seed is not None else s)


def random_circuit(n: int, n_gates: int, seed: int, fixed_fraction: float = 0.3,
                   n_terms: int = 6) -> Problem:
    """A random gate list over all five gate kinds (for small cross-checks).

    Rotations get consecutive parameter indices; fixed gates pick random
    distinct qubit pairs.  The angle/Hamiltonian draw order is the documented
    one, using a second stream (seed + 1) for the gate structure.
    """
    srng = np.random.Generator(np.random.PCG64(seed + 1))
    rows = []
    p = 0
    for _ in range(n_gates):
        if n >= 2 and srng.uniform() < fixed_fraction:
            kind = int(srng.integers(CNOT, CZ + 1))
            a, b = srng.choice(n, size=2, replace=False)
            rows.append([kind, int(a), int(b), -1])
        else:
            kind = int(srng.integers(RX, RZ + 1))
            rows.append([kind, int(srng.integers(0, n)), -1, p])
            p += 1
    gates = np.asarray(rows, dtype=np.int32).reshape(-1, 4)
    theta, pauli, coeff = draw_problem_data(seed, p, n, n_terms)
    return Problem(name=f"random_n{n}_g{n_gates}_s{seed}", n_qubits=n, gates=gates,
                   theta=theta, pauli=pauli, coeff=coeff, seed=seed)


def permute_params(problem: Problem, seed: int) -> Problem:
    """Same circuit with parameter indices relabelled by a random permutation.

    theta is permuted consistently, so the ansatz state is unchanged and G is
    only relabelled.  Used to test that outputs are indexed by parameter.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    P = problem.n_params
    perm = rng.permutation(P)          # old index -> new index
    gates = problem.gates.copy()
    mask = gates[:, 3] >= 0
    gates[mask, 3] = perm[gates[mask, 3]]
    theta = np.empty_like(problem.theta)
    theta[perm] = problem.theta
    return dataclasses.replace(problem, name=problem.name + f"_perm{seed}", gates=gates, theta=theta)


def share_params(problem: Problem, n_shared: int, seed: int) -> Problem:
    """Same circuit with its P parameters merged into n_shared shared ones:
    every parameterised gate is relabelled to one of 0..n_shared-1 (each used at
    least once), with new seeded angles uniform in [0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = problem.n_params
    if not 1 <= n_shared <= P:
        raise ValueError("need 1 <= n_shared <= P")
    labels = np.concatenate([np.arange(n_shared), rng.integers(0, n_shared, P - n_shared)])
    rng.shuffle(labels)                 # old parameter -> shared parameter
    gates = problem.gates.copy()
    mask = gates[:, 3] >= 0
    gates[mask, 3] = labels[gates[mask, 3]]
    theta = rng.uniform(0.0, 2.0 * np.pi, n_shared)
    return dataclasses.replace(problem, name=problem.name + f"_shared{n_shared}", gates=gates, theta=theta)


def layer_shared(n: int, layers: int, n_terms: int, seed: int) -> Problem:
    """Layers of RX on every qubit (one angle per layer), a CNOT chain and RZ on
    every qubit (one angle per layer): 2 parameters per layer, each carried by
    n gates.  Seeded angles and Pauli-sum Hamiltonian as in the other workloads."""
    base = make_problem(f"layer_shared_n{n}_L{layers}", n, layers, (RX, RZ), "cnot_chain", n_terms, seed)
    gates = base.gates.copy()
    rot = np.nonzero(gates[:, 3] >= 0)[0]
    per_layer = 2 * n
    for k, g in enumerate(rot):
        layer, within = divmod(k, per_layer)
        gates[g, 3] = 2 * layer + (0 if within < n else 1)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    theta = rng.uniform(0.0, 2.0 * np.pi, 2 * layers)
    return dataclasses.replace(base, gates=gates, theta=theta)


def controlled_circuit(n: int, n_gates: int, seed: int, controlled_fraction: float = 0.35,
                       fixed_fraction: float = 0.2, n_terms: int = 6) -> Problem:
    """A random gate list with controlled rotations among the other kinds.

    Each gate is, in this order of draws from a second stream (seed + 1): a
    fixed two-qubit gate (CNOT/CZ) with probability ``fixed_fraction``, else a
    controlled rotation (CRX/CRY/CRZ on a random distinct control/target pair)
    with probability ``controlled_fraction``, else a plain rotation.  Every
    parameterised gate gets the next parameter index; angles and Hamiltonian
    follow the documented draw order from ``seed``.
    """
    assert n >= 2
    srng = np.random.Generator(np.random.PCG64(seed + 1))
    rows = []
    p = 0
    for _ in range(n_gates):
        u = srng.uniform()
        if u < fixed_fraction:
            kind = int(srng.integers(CNOT, CZ + 1))
            a, b = srng.choice(n, size=2, replace=False)
            rows.append([kind, int(a), int(b), -1])
        elif u < fixed_fraction + controlled_fraction:
            kind = int(srng.integers(CRX, CRZ + 1))
            a, b = srng.choice(n, size=2, replace=False)
            rows.append([kind, int(a), int(b), p])
            p += 1
        else:
            rows.append([int(srng.integers(RX, RZ + 1)), int(srng.integers(0, n)), -1, p])
            p += 1
    gates = np.asarray(rows, dtype=np.int32).reshape(-1, 4)
    theta, pauli, coeff = draw_problem_data(seed, p, n, n_terms)
    return Problem(name=f"controlled_n{n}_g{n_gates}_s{seed}", n_qubits=n, gates=gates,
                   theta=theta, pauli=pauli, coeff=coeff, seed=seed)


def controlled_layers(n: int, layers: int, n_terms: int, seed: int, dt: float = 0.1,
                      tikhonov: float = 1e-4) -> Problem:
    """Layers of [RY on every qubit, then CRZ(q -> q+1) for q = 0..n-2, then
    CRX(n-1 -> 0)]: a ring of controlled rotations, each with its own angle
    (P = layers * 2n).  Angles and Hamiltonian in the documented draw order."""
    rows: List[List[int]] = []
    p = 0
    for _ in range(layers):
        for q in range(n):
            rows.append([RY, q, -1, p])
            p += 1
        for q in range(n - 1):
            rows.append([CRZ, q, q + 1, p])
            p += 1
        rows.append([CRX, n - 1, 0, p])
        p += 1
    gates = np.asarray(rows, dtype=np.int32).reshape(-1, 4)
    theta, pauli, coeff = draw_problem_data(seed, p, n, n_terms)
    return Problem(name=f"controlled_layers_n{n}_L{layers}", n_qubits=n, gates=gates, theta=theta,
                   pauli=pauli, coeff=coeff, dt=dt, tikhonov=tikhonov, seed=seed)


def string_circuit(n: int, n_gates: int, seed: int, string_fraction: float = 0.4,
                   fixed_fraction: float = 0.2, max_support: int = 4, n_terms: int = 6) -> Problem:
    """A random gate list with Pauli-string rotations among the other kinds.

    Each gate is, in this order of draws from a second stream (seed + 1): a
    fixed gate (CNOT/CZ) with probability ``fixed_fraction``, else a
    Pauli-string rotation with probability ``string_fraction`` -- its support
    is a random set of 1..min(n, max_support) qubits, each carrying a letter
    drawn from {X, Y, Z}, and it adds a row to ``strings`` -- else a plain
    rotation.  Angles and Hamiltonian follow the documented draw order.
    """
    srng = np.random.Generator(np.random.PCG64(seed + 1))
    rows, strings = [], []
    p = 0
    for _ in range(n_gates):
        u = srng.uniform()
        if n >= 2 and u < fixed_fraction:
            kind = int(srng.integers(CNOT, CZ + 1))
            a, b = srng.choice(n, size=2, replace=False)
            rows.append([kind, int(a), int(b), -1])
        elif u < fixed_fraction + string_fraction:
            k = int(srng.integers(1, min(n, max_support) + 1))
            support = srng.choice(n, size=k, replace=False)
            letters = np.zeros(n, dtype=np.uint8)
            letters[support] = srng.integers(1, 4, size=k)
            rows.append([RPAULI, len(strings), -1, p])
            strings.append(letters)
            p += 1
        else:
            rows.append([int(srng.integers(RX, RZ + 1)), int(srng.integers(0, n)), -1, p])
            p += 1
    gates = np.asarray(rows, dtype=np.int32).reshape(-1, 4)
    theta, pauli, coeff = draw_problem_data(seed, p, n, n_terms)
    table = np.asarray(strings, dtype=np.uint8).reshape(-1, n)
    return Problem(name=f"strings_n{n}_g{n_gates}_s{seed}", n_qubits=n, gates=gates, theta=theta, pauli=pauli,
                   coeff=coeff, seed=seed, strings=table)


def string_layers(n: int, layers: int, n_terms: int, seed: int, dt: float = 0.1, tikhonov: float = 1e-4) -> Problem:
    """Layers of [RX on every qubit, then ZZ rotations exp(i t Z_q Z_{q+1}/2) for
    q = 0..n-2, then one rotation about X Y ... Y X on every qubit (X at both
    ends)]: P = layers * 2n.  Angles and Hamiltonian in the documented draw order."""
    strings = []
    for q in range(n - 1):
        s_ = np.zeros(n, dtype=np.uint8)
        s_[q] = s_[q + 1] = 3
        strings.append(s_)
    ladder = np.full(n, 2, dtype=np.uint8)
    ladder[0] = ladder[n - 1] = 1
    strings.append(ladder)
    rows: List[List[int]] = []
    p = 0
    for _ in range(layers):
        for q in range(n):
            rows.append([RX, q, -1, p])
            p += 1
        for k in range(n):
            rows.append([RPAULI, k, -1, p])
            p += 1
    gates = np.asarray(rows, dtype=np.int32).reshape(-1, 4)
    theta, pauli, coeff = draw_problem_data(seed, p, n, n_terms)
    return Problem(name=f"string_layers_n{n}_L{layers}", n_qubits=n, gates=gates, theta=theta, pauli=pauli,
                   coeff=coeff, dt=dt, tikhonov=tikhonov, seed=seed, strings=np.asarray(strings, dtype=np.uint8))


def random_state(n: int, seed: int) -> np.ndarray:
    """A normalised random complex128 input state (Gaussian amplitudes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    return (v / np.linalg.norm(v)).astype(np.complex128)
