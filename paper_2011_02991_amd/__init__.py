"""Python binding of libqng (include/qng.h): argument marshalling only.

Every step of the quantum-natural-gradient path runs inside the HIP library;
this module converts numpy arrays / torch tensors into the plain pointers and
sizes of the C ABI and turns status codes into exceptions.  If the built
library is missing, importing the binding raises: there is no fallback.

Problems are described the way the library's C ABI describes them: a gate
list of rows (kind, q0, q1, param) with kind 0/1/2 = RX/RY/RZ (rotation
exp(+i theta sigma/2)), 3 = CNOT (control q0, target q1), 4 = CZ, 5/6/7 =
controlled RX/RY/RZ (control q0, target q1), 8 = Pauli-string rotation (q0 =
row of a table of letters per qubit); a vector of
angles indexed by parameter; a Pauli-sum Hamiltonian (letters 0..3 = I, X, Y, Z
per qubit, real coefficients); an optional complex128 input state.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqng.so")

C128, C64 = 0, 1
PRECISIONS = {"c128": C128, "complex128": C128, C128: C128, "c64": C64, "complex64": C64, C64: C64}

OPT_FUSION, OPT_TILE_QUBITS, OPT_COLUMN_STREAMS, OPT_PROFILE, OPT_SMALL_N_KERNEL, OPT_F64_REGISTERS = 0, 1, 2, 3, 4, 5
OPT_GRAPH, OPT_AUTOTUNE, OPT_BATCH_TILES, OPT_BLOCK_COLUMNS, OPT_METRIC_KIND, OPT_EXACT_PRODUCTS = 6, 7, 8, 9, 10, 11
OPT_METHOD = 12
OPT_STATE_CHUNK = 13

STATUS = {
    0: "QNG_OK", -1: "QNG_E_INVALID_ARG", -2: "QNG_E_BAD_CIRCUIT", -3: "QNG_E_BAD_PARAMS",
    -4: "QNG_E_NOT_NORMALIZED", -5: "QNG_E_NONFINITE", -6: "QNG_E_OUT_OF_MEMORY", -7: "QNG_E_NOT_SPD",
    -8: "QNG_E_DEVICE", -9: "QNG_E_UNSUPPORTED",
}


class QNGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class _Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32), ("param", ctypes.c_int32)]


class _Circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32), ("n_params", ctypes.c_int32),
                ("gates", ctypes.c_void_p), ("n_strings", ctypes.c_int32), ("strings", ctypes.c_void_p)]


class _PauliSum(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("coeff", ctypes.c_void_p), ("pauli", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("sweep_launches", ctypes.c_int64), ("sweep_tiles", ctypes.c_int64), ("sweep_ms", ctypes.c_double),
                ("sweep_bytes", ctypes.c_double), ("sweep_flops", ctypes.c_double), ("elements", ctypes.c_int64), ("other_launches", ctypes.c_int64),
                ("metric_ms", ctypes.c_double), ("grad_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("tile_qubits", ctypes.c_int32), ("target_tiles", ctypes.c_int32), ("tune_ms", ctypes.c_double),
                ("graph_replays", ctypes.c_int64), ("block_columns", ctypes.c_int32), ("state_chunks", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanInfo(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int64), ("elements", ctypes.c_int64), ("ops", ctypes.c_int64),
                ("transposes", ctypes.c_int64), ("tile_qubits", ctypes.c_int32), ("small_n", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libqng.so is not built ({LIB_PATH}); run __graft_entry__.build() or "
                          f"python paper_2011_02991_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    sigs = {
        "qng_create": [vp, ctypes.c_int, vp],
        "qng_destroy": [vp],
        "qng_last_error": [vp],
        "qng_set_stream": [vp, vp],
        "qng_set_mem_limit": [vp, sz],
        "qng_set_option": [vp, ctypes.c_int, ctypes.c_int],
        "qng_set_metric_blocks": [vp, i32, vp],
        "qng_get_stats": [vp, vp],
        "qng_synchronize": [vp],
        "qng_validate": [vp, vp, vp, ctypes.c_char_p, sz],
        "qng_plan": [vp, ctypes.c_int, ctypes.c_int, vp],
        "qng_solve_shifted": [i32, vp, dbl, vp, vp],
        "qng_metric": [vp, vp, vp, vp, ctypes.c_int, vp, vp],
        "qng_energy_grad": [vp, vp, vp, vp, vp, ctypes.c_int, vp, vp],
        "qng_step": [vp, vp, vp, vp, vp, dbl, dbl, ctypes.c_int, vp, vp, vp, vp],
        "qng_step_batched": [vp, i32, vp, vp, vp, vp, dbl, dbl, ctypes.c_int, vp, vp, vp, vp],
        "qng_metric_dev": [vp, vp, vp, vp, ctypes.c_int, vp, vp],
        "qng_energy_dev": [vp, vp, vp, vp, vp, ctypes.c_int, vp, vp],
        "qng_energy_grad_from_state_dev": [vp, vp, vp, vp, ctypes.c_int, vp, vp],
        "qng_apply_circuit_dev": [vp, vp, vp, ctypes.c_int, vp],
        "qng_energy_grad_dev": [vp, vp, vp, vp, vp, ctypes.c_int, vp, vp],
        "qng_step_dev": [vp, vp, vp, vp, vp, dbl, dbl, ctypes.c_int, vp, vp, vp, vp, vp],
        "qng_clone_state_dev": [vp, i32, ctypes.c_int, vp, vp],
        "qng_energy_grad_dev_noalloc": [vp, vp, vp, vp, vp, ctypes.c_int, vp, vp],
        "qng_plan_export": [vp, ctypes.c_int, ctypes.c_int, i32, vp, ctypes.c_int64, vp],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.qng_destroy.restype = None
    lib.qng_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()

# Symbols the C header declares (checked by the CPU test suite).
EXPORTED = ("qng_create", "qng_destroy", "qng_last_error", "qng_set_stream", "qng_set_mem_limit", "qng_set_option",
            "qng_set_metric_blocks",
            "qng_get_stats", "qng_synchronize", "qng_validate", "qng_plan", "qng_solve_shifted", "qng_metric",
            "qng_energy_grad", "qng_step", "qng_step_batched", "qng_metric_dev", "qng_energy_dev",
            "qng_energy_grad_from_state_dev", "qng_apply_circuit_dev", "qng_plan_export", "qng_energy_grad_dev",
            "qng_step_dev", "qng_clone_state_dev", "qng_energy_grad_dev_noalloc")


def lib():
    return _lib


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    return a.ctypes.data


def _check(status: int, ctx=None):
    if status != 0:
        msg = _lib.qng_last_error(ctx)
        raise QNGError(status, msg.decode() if msg else "")


def _prec(p) -> int:
    if p not in PRECISIONS:
        raise ValueError(f"unknown precision {p!r}")
    return PRECISIONS[p]


class Circuit:
    """Marshalled circuit (+ optional Hamiltonian) kept alive for the C calls."""

    def __init__(self, n_qubits: int, gates, n_params: Optional[int] = None, pauli=None, coeff=None,
                 strings=None):
        self.gates = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 4))
        self.n_qubits = int(n_qubits)
        self.n_params = int((self.gates[:, 3] >= 0).sum()) if n_params is None else int(n_params)
        # letters of the Pauli-string rotations (kind 8): one row of n_qubits per string
        self.strings = (np.zeros((0, self.n_qubits), dtype=np.uint8) if strings is None else
                        np.ascontiguousarray(np.asarray(strings, dtype=np.uint8).reshape(-1, self.n_qubits)))
        self.c = _Circuit(self.n_qubits, self.gates.shape[0], self.n_params,
                          self.gates.ctypes.data if self.gates.size else None, self.strings.shape[0],
                          self.strings.ctypes.data if self.strings.size else None)
        self.h = None
        if pauli is not None:
            self.pauli = np.ascontiguousarray(np.asarray(pauli, dtype=np.uint8).reshape(-1, self.n_qubits))
            self.coeff = np.ascontiguousarray(np.asarray(coeff, dtype=np.float64))
            self.h = _PauliSum(self.coeff.shape[0], self.coeff.ctypes.data if self.coeff.size else None,
                               self.pauli.ctypes.data if self.pauli.size else None)

    @classmethod
    def from_problem(cls, pr) -> "Circuit":
        return cls(pr.n_qubits, pr.gates, pr.n_params, pr.pauli, pr.coeff, getattr(pr, "strings", None))

    @property
    def cref(self):
        return ctypes.byref(self.c)

    @property
    def href(self):
        if self.h is None:
            raise ValueError("circuit has no Hamiltonian")
        return ctypes.byref(self.h)


def _theta(theta) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(theta, dtype=np.float64))


def _in_state(s) -> Optional[np.ndarray]:
    if s is None:
        return None
    return np.ascontiguousarray(np.asarray(s, dtype=np.complex128))


def validate(circ: Circuit, theta, with_hamiltonian: bool = True) -> None:
    """Host-only validation (no GPU).  Raises QNGError."""
    th = _theta(theta)
    buf = ctypes.create_string_buffer(512)
    st = _lib.qng_validate(circ.cref, _ptr(th), circ.href if (with_hamiltonian and circ.h is not None) else None,
                           buf, 512)
    if st != 0:
        raise QNGError(st, buf.value.decode())


def plan(circ: Circuit, fusion: int = 1, tile_qubits: int = 0) -> dict:
    """Host-only compile of the sweep plan; returns its size."""
    info = PlanInfo()
    _check(_lib.qng_plan(circ.cref, fusion, tile_qubits, ctypes.byref(info)))
    return info.as_dict()


def plan_export(circ: Circuit, tile_qubits: int = 0, prec="c128", gradient: bool = False,
                block: int = 1) -> np.ndarray:
    """Host-only: a fused sweep plan as rows of 10 int32 (see qng_plan_export);
    the metric's columns (block=2 or 4: that many columns per lambda sweep), or
    the gradient's reverse sweep."""
    amp = 16 if _prec(prec) == C128 else 8
    if block not in (1, 2, 4):
        raise ValueError("block must be 1, 2 or 4")
    sw = 1 if gradient else (block if block > 1 else 0)
    n = ctypes.c_int64()
    _check(_lib.qng_plan_export(circ.cref, tile_qubits, amp, sw, None, 0, ctypes.byref(n)))
    rows = np.zeros((n.value, 10), dtype=np.int32)
    _check(_lib.qng_plan_export(circ.cref, tile_qubits, amp, sw, _ptr(rows), n.value, ctypes.byref(n)))
    return rows


def solve_shifted(G: np.ndarray, eps: float, b: np.ndarray) -> np.ndarray:
    G = np.ascontiguousarray(G, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty_like(b)
    _check(_lib.qng_solve_shifted(b.shape[0], _ptr(G), float(eps), _ptr(b), _ptr(x)))
    return x


class Context:
    """A library context on one HIP device (owns the device workspace)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        h = ctypes.c_void_p()
        _check(_lib.qng_create(ctypes.byref(h), int(device), stream))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.qng_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, st):
        _check(st, self._h)

    def set_option(self, option: int, value: int):
        self._c(_lib.qng_set_option(self._h, option, int(value)))

    def set_metric_blocks(self, block_of_param=None):
        """Block-diagonal metric: block id per parameter (None clears it)."""
        if block_of_param is None:
            self._c(_lib.qng_set_metric_blocks(self._h, 0, None))
            return
        b = np.ascontiguousarray(block_of_param, dtype=np.int32)
        self._c(_lib.qng_set_metric_blocks(self._h, int(b.shape[0]), _ptr(b)))

    def set_stream(self, stream: Optional[int]):
        self._c(_lib.qng_set_stream(self._h, stream))

    def set_mem_limit(self, nbytes: int):
        self._c(_lib.qng_set_mem_limit(self._h, int(nbytes)))

    def synchronize(self):
        self._c(_lib.qng_synchronize(self._h))

    def stats(self) -> dict:
        s = Stats()
        self._c(_lib.qng_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    # ---------------------------------------------------------------- host API
    def metric(self, circ: Circuit, theta, in_state=None, prec="c128"):
        th, ins = _theta(theta), _in_state(in_state)
        P = circ.n_params
        G = np.zeros((P, P), dtype=np.complex128)
        T = np.zeros(P, dtype=np.complex128)
        self._c(_lib.qng_metric(self._h, circ.cref, _ptr(ins), _ptr(th), _prec(prec), _ptr(G), _ptr(T)))
        return G, T

    def energy_grad(self, circ: Circuit, theta, in_state=None, prec="c128"):
        th, ins = _theta(theta), _in_state(in_state)
        E = np.zeros(1)
        grad = np.zeros(circ.n_params)
        self._c(_lib.qng_energy_grad(self._h, circ.cref, _ptr(ins), circ.href, _ptr(th), _prec(prec), _ptr(E),
                                     _ptr(grad)))
        return float(E[0]), grad

    def step(self, circ: Circuit, theta, dt: float, tikhonov: float, in_state=None, prec="c128",
             want_G: bool = True):
        th, ins = _theta(theta), _in_state(in_state)
        P = circ.n_params
        dth = np.zeros(P)
        G = np.zeros((P, P), dtype=np.complex128) if want_G else None
        grad = np.zeros(P)
        E = np.zeros(1)
        self._c(_lib.qng_step(self._h, circ.cref, _ptr(ins), circ.href, _ptr(th), float(dt), float(tikhonov),
                              _prec(prec), _ptr(dth), _ptr(G), _ptr(grad), _ptr(E)))
        return {"dtheta": dth, "G": G, "grad": grad, "E": float(E[0])}

    def step_batched(self, circs: Sequence[Circuit], thetas, dt: float, tikhonov: float, in_states=None,
                     prec="c128", want_G: bool = True):
        B = len(circs)
        carr = (_Circuit * B)(*[c.c for c in circs])
        harr = (_PauliSum * B)(*[c.h for c in circs])
        ths = [_theta(t) for t in thetas]
        ins = [_in_state(s) for s in in_states] if in_states is not None else [None] * B
        outs = [np.zeros(c.n_params) for c in circs]
        Gs = [np.zeros((c.n_params, c.n_params), dtype=np.complex128) for c in circs] if want_G else None
        grads = [np.zeros(c.n_params) for c in circs]
        E = np.zeros(B)
        P = ctypes.c_void_p
        mk = lambda arrs: (P * B)(*[_ptr(a) for a in arrs])
        self._c(_lib.qng_step_batched(self._h, B, carr, mk(ins), harr, mk(ths), float(dt), float(tikhonov),
                                      _prec(prec), mk(outs), mk(Gs) if want_G else None, mk(grads), _ptr(E)))
        return [{"dtheta": outs[b], "G": Gs[b] if want_G else None, "grad": grads[b], "E": float(E[b])}
                for b in range(B)]

    # -------------------------------------------------------------- device API
    def metric_dev(self, circ: Circuit, theta, G_dev_ptr: int, T_dev_ptr: Optional[int] = None,
                   in_state_dev_ptr: Optional[int] = None, prec="c128"):
        th = _theta(theta)
        self._c(_lib.qng_metric_dev(self._h, circ.cref, in_state_dev_ptr, _ptr(th), _prec(prec), G_dev_ptr,
                                    T_dev_ptr))

    def energy_dev(self, circ: Circuit, theta, E_dev_ptr: int, psi_dev_ptr: int,
                   in_state_dev_ptr: Optional[int] = None, prec="c128"):
        th = _theta(theta)
        self._c(_lib.qng_energy_dev(self._h, circ.cref, in_state_dev_ptr, circ.href, _ptr(th), _prec(prec),
                                    E_dev_ptr, psi_dev_ptr))

    def apply_circuit_dev(self, circ: Circuit, theta, state_dev_ptr: int, prec="c128"):
        th = _theta(theta)
        self._c(_lib.qng_apply_circuit_dev(self._h, circ.cref, _ptr(th) if th.size else None, _prec(prec),
                                           state_dev_ptr))

    def energy_grad_dev(self, circ: Circuit, theta, E_dev_ptr: int, grad_dev_ptr: int,
                        in_state_dev_ptr: Optional[int] = None, prec="c128"):
        th = _theta(theta)
        self._c(_lib.qng_energy_grad_dev(self._h, circ.cref, in_state_dev_ptr, circ.href, _ptr(th), _prec(prec),
                                         E_dev_ptr, grad_dev_ptr))

    def energy_grad_dev_noalloc(self, circ: Circuit, theta, E_dev_ptr: int, grad_dev_ptr: int,
                                in_state_dev_ptr: Optional[int] = None, prec="c128"):
        th = _theta(theta)
        self._c(_lib.qng_energy_grad_dev_noalloc(self._h, circ.cref, in_state_dev_ptr, circ.href, _ptr(th),
                                                 _prec(prec), E_dev_ptr, grad_dev_ptr))

    def step_dev(self, circ: Circuit, theta, dt: float, tikhonov: float, dtheta_dev_ptr: int,
                 G_dev_ptr: Optional[int] = None, grad_dev_ptr: Optional[int] = None, E_dev_ptr: Optional[int] = None,
                 status_dev_ptr: Optional[int] = None, in_state_dev_ptr: Optional[int] = None, prec="c128"):
        th = _theta(theta)
        self._c(_lib.qng_step_dev(self._h, circ.cref, in_state_dev_ptr, circ.href, _ptr(th), float(dt),
                                  float(tikhonov), _prec(prec), dtheta_dev_ptr, G_dev_ptr, grad_dev_ptr, E_dev_ptr,
                                  status_dev_ptr))

    def clone_state_dev(self, n_qubits: int, src_dev_ptr: int, dst_dev_ptr: int, prec="c128"):
        self._c(_lib.qng_clone_state_dev(self._h, int(n_qubits), _prec(prec), src_dev_ptr, dst_dev_ptr))

    def energy_grad_from_state_dev(self, circ: Circuit, theta, psi_dev_ptr: int, grad_dev_ptr: int, prec="c128"):
        th = _theta(theta)
        self._c(_lib.qng_energy_grad_from_state_dev(self._h, circ.cref, circ.href, _ptr(th), _prec(prec),
                                                    psi_dev_ptr, grad_dev_ptr))
