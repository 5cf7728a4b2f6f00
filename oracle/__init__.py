"""Python access to the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It takes
the symbolic gate lists of :mod:`circuits` and hands them to the C oracle
using the oracle's own gate numbering; it imports nothing from the HIP path.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KINDS = {"H": 1, "X": 2, "Y": 3, "Z": 4, "S": 5, "T": 6,
         "RX": 7, "RY": 8, "RZ": 9, "U1": 10, "U": 11}
MAXK = 6

_c_cplx_p = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_c_f64_p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_c_i32_p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_c_i64_p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_c_u64_p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (C11, OpenMP) into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.oc_init_basis.argtypes = [ctypes.c_int, ctypes.c_uint64, _c_cplx_p]
        L.oc_gate_matrix.argtypes = [ctypes.c_int, ctypes.c_double, _c_cplx_p]
        L.oc_gate_matrix.restype = ctypes.c_int
        L.oc_gate_dmatrix.argtypes = [ctypes.c_int, ctypes.c_double, _c_cplx_p]
        L.oc_gate_dmatrix.restype = ctypes.c_int
        L.oc_apply_1q.argtypes = [ctypes.c_int, _c_cplx_p, ctypes.c_int, ctypes.c_uint64, _c_cplx_p]
        L.oc_apply_kq.argtypes = [ctypes.c_int, _c_cplx_p, ctypes.c_int, _c_i32_p,
                                  ctypes.c_uint64, _c_cplx_p]
        L.oc_run.argtypes = [ctypes.c_int, _c_cplx_p, ctypes.c_int, _c_i32_p, _c_i32_p, _c_u64_p,
                             _c_f64_p, _c_i64_p, _c_cplx_p, ctypes.c_int]
        L.oc_probabilities.argtypes = [ctypes.c_int, _c_cplx_p, _c_f64_p]
        L.oc_probabilities.restype = ctypes.c_double
        L.oc_expectation_z.argtypes = [ctypes.c_int, _c_cplx_p, ctypes.c_int, _c_u64_p, _c_f64_p]
        L.oc_expectation_z.restype = ctypes.c_double
        L.oc_adjoint_grad.argtypes = [ctypes.c_int, _c_cplx_p, _c_cplx_p, _c_cplx_p, ctypes.c_int,
                                      _c_i32_p, _c_i32_p, _c_u64_p, _c_f64_p, _c_i32_p, _c_i64_p,
                                      _c_cplx_p, _c_f64_p, ctypes.c_int, ctypes.c_int, _c_u64_p,
                                      _c_f64_p, _c_f64_p]
        L.oc_adjoint_grad.restype = ctypes.c_double
        L.oc_marginals.argtypes = [ctypes.c_int, _c_cplx_p, ctypes.c_uint64, _c_f64_p]
        L.oc_collapse.argtypes = [ctypes.c_int, _c_cplx_p, ctypes.c_uint64, ctypes.c_uint64]
        L.oc_collapse.restype = ctypes.c_double
        L.oc_select.argtypes = [ctypes.c_uint64, _c_f64_p, ctypes.c_double]
        L.oc_select.restype = ctypes.c_uint64
        L.oc_sample.argtypes = [ctypes.c_int, _c_cplx_p, ctypes.c_int, _c_f64_p, _c_u64_p]
        L.oc_measure.argtypes = [ctypes.c_int, _c_cplx_p, ctypes.c_uint64, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_uint64)]
        L.oc_measure.restype = ctypes.c_double
        L.oc_num_threads.restype = ctypes.c_int
        L.oc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oc_num_threads())


def set_num_threads(t: int) -> None:
    """Host threads of the following oracle calls (t < 1: the default)."""
    lib().oc_set_num_threads(int(t))


class _Packed:
    """A gate list in the oracle's array form."""

    def __init__(self, gates):
        g = len(gates)
        self.n_gates = g
        self.kind = np.zeros(max(g, 1), np.int32)
        self.tq = np.full(max(g, 1) * MAXK, -1, np.int32)
        self.ctrl = np.zeros(max(g, 1), np.uint64)
        self.theta = np.zeros(max(g, 1), np.float64)
        self.param = np.full(max(g, 1), -1, np.int32)
        self.mat_off = np.zeros(max(g, 1), np.int64)
        mats: List[np.ndarray] = []
        off = 0
        for i, gt in enumerate(gates):
            self.kind[i] = KINDS[gt.name]
            if len(gt.targets) > MAXK:
                raise ValueError("oracle takes at most 6 target qubits")
            for j, q in enumerate(gt.targets):
                self.tq[i * MAXK + j] = q
            m = 0
            for c in gt.controls:
                m |= 1 << c
            self.ctrl[i] = m
            self.theta[i] = gt.theta
            self.param[i] = gt.param
            if gt.name == "U":
                mm = np.ascontiguousarray(gt.matrix, dtype=np.complex128).reshape(-1)
                if mm.size != (1 << (2 * len(gt.targets))):
                    raise ValueError("matrix size does not match the target count")
                self.mat_off[i] = off
                mats.append(mm)
                off += mm.size
            elif len(gt.targets) != 1:
                raise ValueError(f"{gt.name} is a one-qubit gate")
        self.mats = np.concatenate(mats) if mats else np.zeros(1, np.complex128)


def basis_state(n: int, x: int = 0) -> np.ndarray:
    psi = np.empty(1 << n, np.complex128)
    lib().oc_init_basis(n, x, psi)
    return psi


def gate_matrix(name: str, theta: float = 0.0) -> np.ndarray:
    m = np.empty(4, np.complex128)
    if lib().oc_gate_matrix(KINDS[name], theta, m) != 0:
        raise ValueError(name)
    return m.reshape(2, 2)


def gate_dmatrix(name: str, theta: float) -> np.ndarray:
    m = np.empty(4, np.complex128)
    if lib().oc_gate_dmatrix(KINDS[name], theta, m) != 0:
        raise ValueError(name)
    return m.reshape(2, 2)


def apply_1q(psi: np.ndarray, n: int, t: int, m: np.ndarray, ctrl: int = 0) -> None:
    lib().oc_apply_1q(n, psi, t, ctrl, np.ascontiguousarray(m, np.complex128).reshape(-1))


def apply_kq(psi: np.ndarray, n: int, qubits: Sequence[int], m: np.ndarray, ctrl: int = 0) -> None:
    q = np.asarray(qubits, np.int32)
    lib().oc_apply_kq(n, psi, len(q), q, ctrl, np.ascontiguousarray(m, np.complex128).reshape(-1))


def run(circuit, psi: Optional[np.ndarray] = None, inverse: bool = False) -> np.ndarray:
    """Final state of ``circuit`` (from |circuit.basis> unless psi is given;
    psi is updated in place)."""
    c = circuit.bound()
    if psi is None:
        psi = basis_state(c.n, c.basis)
    p = _Packed(c.gates)
    lib().oc_run(c.n, psi, p.n_gates, p.kind, p.tq, p.ctrl, p.theta, p.mat_off, p.mats,
                 1 if inverse else 0)
    return psi


def run_gates(n: int, gates, psi: np.ndarray, inverse: bool = False) -> np.ndarray:
    p = _Packed(gates)
    lib().oc_run(n, psi, p.n_gates, p.kind, p.tq, p.ctrl, p.theta, p.mat_off, p.mats,
                 1 if inverse else 0)
    return psi


def probabilities(psi: np.ndarray, n: int) -> Tuple[np.ndarray, float]:
    p = np.empty(1 << n, np.float64)
    total = lib().oc_probabilities(n, psi, p)
    return p, float(total)


def expectation_z(psi: np.ndarray, n: int, masks: Sequence[int], coeffs: Sequence[float]) -> float:
    m = np.asarray(masks, np.uint64)
    c = np.asarray(coeffs, np.float64)
    return float(lib().oc_expectation_z(n, psi, len(m), m, c))


def marginals(psi: np.ndarray, n: int, mask: int) -> np.ndarray:
    """Outcome probabilities of the qubits of mask (Sec. 1.3.3)."""
    out = np.empty(1 << bin(mask).count("1"), np.float64)
    lib().oc_marginals(n, psi, mask, out)
    return out


def collapse(psi: np.ndarray, n: int, mask: int, value: int) -> float:
    """Project psi (in place) onto (x & mask) == (value & mask), renormalise; returns p."""
    return float(lib().oc_collapse(n, psi, mask, value))


def select(p: np.ndarray, u: float) -> int:
    """Inverse-CDF outcome selection over the outcome probabilities p."""
    p = np.ascontiguousarray(p, np.float64)
    return int(lib().oc_select(len(p), p, u))


def sample(psi: np.ndarray, n: int, uniforms) -> np.ndarray:
    """Full-register outcomes for the given uniforms in [0, 1); psi unchanged."""
    u = np.ascontiguousarray(uniforms, np.float64)
    out = np.empty(len(u), np.uint64)
    lib().oc_sample(n, psi, len(u), u, out)
    return out


def measure(psi: np.ndarray, n: int, mask: int, u: float) -> Tuple[int, float]:
    """Measure the qubits of mask with uniform u; psi collapses in place.
    Returns (outcome bits at the mask positions, probability)."""
    v = ctypes.c_uint64()
    p = lib().oc_measure(n, psi, mask, u, ctypes.byref(v))
    return int(v.value), float(p)


def loss(circuit, params: np.ndarray, masks, coeffs) -> float:
    c = circuit.bound() if params is None else type(circuit)(
        circuit.n, circuit.gates, circuit.basis, np.asarray(params, np.float64), circuit.name).bound()
    psi = run(c)
    return expectation_z(psi, c.n, masks, coeffs)


def adjoint_grad(circuit, params: np.ndarray, masks, coeffs) -> Tuple[float, np.ndarray]:
    n = circuit.n
    p = _Packed(circuit.gates)
    params = np.ascontiguousarray(params, np.float64)
    grad = np.zeros(len(params), np.float64)
    psi = np.empty(1 << n, np.complex128)
    lam = np.empty(1 << n, np.complex128)
    mu = np.empty(1 << n, np.complex128)
    m = np.asarray(masks, np.uint64)
    cf = np.asarray(coeffs, np.float64)
    L = lib().oc_adjoint_grad(n, psi, lam, mu, p.n_gates, p.kind, p.tq, p.ctrl, p.theta, p.param,
                              p.mat_off, p.mats, params, len(params), len(m), m, cf, grad)
    return float(L), grad
