"""MI355X (gfx950) state-vector simulator: Python binding of libsv.so.

Functions named after the C entry points marshal arguments (torch tensors
for device memory and the current HIP stream, numpy arrays for host data)
and call the library; every step of the simulation runs in the library's HIP
kernels.  :class:`State` bundles a register's device buffer and handle.
There is no CPU fallback: without the built library every call raises.
"""

from __future__ import annotations

import ctypes
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import (GATE_KINDS, SV_C64, SV_C128, SV_PREC_FP32, SV_PREC_NATIVE,
                   SV_PREC_SPLIT_BF16, SV_RUN_PER_GATE, SV_RUN_TILED, SVError, sv_op)

__all__ = ["State", "sv_alloc", "sv_free", "sv_set_basis", "sv_apply_gate", "sv_apply_fused",
           "sv_probabilities", "sv_expectation", "sv_expectation_noalloc", "sv_run", "sv_schedule", "sv_fuse", "sv_run_fused", "sv_fused_tune",
           "sv_adjoint_grad", "sv_state_bytes", "ops_from_gates", "SV_C64", "SV_C128",
           "SV_PREC_NATIVE", "SV_PREC_FP32", "SV_PREC_SPLIT_BF16", "SV_RUN_PER_GATE",
           "SV_RUN_TILED", "SVError", "Batch"]


def _torch():
    import torch
    return torch


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _u64ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _current_stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dtype_code(dtype) -> int:
    if dtype in (SV_C64, SV_C128):
        return dtype
    torch = _torch()
    if dtype in ("c64", "complex64", torch.complex64, np.complex64):
        return SV_C64
    if dtype in ("c128", "complex128", torch.complex128, np.complex128):
        return SV_C128
    raise ValueError(f"unsupported dtype {dtype!r}")


# ------------------------------------------------------------ C-ABI mirrors

def sv_state_bytes(n_qubits: int, dtype) -> int:
    return int(_lib.load().sv_state_bytes(n_qubits, _dtype_code(dtype)))


def sv_alloc(n_qubits: int, dtype, dev_buf=None, stream=None) -> ctypes.c_void_p:
    """Handle of an n-qubit register in |0..0>.  dev_buf: a CUDA tensor of
    2^n complex elements to use as storage (kept alive by the caller)."""
    h = ctypes.c_void_p()
    ptr = ctypes.c_void_p(dev_buf.data_ptr()) if dev_buf is not None else None
    s = stream if stream is not None else _current_stream()
    _lib.check(_lib.load().sv_alloc(n_qubits, _dtype_code(dtype), ptr, s, ctypes.byref(h)))
    return h


def sv_free(h) -> None:
    _lib.check(_lib.load().sv_free(h))


def sv_set_basis(h, x: int) -> None:
    _lib.check(_lib.load().sv_set_basis(h, int(x)))


def sv_sync(h) -> None:
    _lib.check(_lib.load().sv_sync(h))


def _mat(U) -> np.ndarray:
    U = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
    return np.ascontiguousarray(U.view(np.float64).reshape(-1))


def sv_apply_gate(h, targets: Sequence[int], U, ctrl_mask: int = 0) -> None:
    t = np.ascontiguousarray(targets, dtype=np.int32)
    m = _mat(U)
    _lib.check(_lib.load().sv_apply_gate(h, len(t), _iptr(t), int(ctrl_mask), _dptr(m)))


def sv_apply_fused(h, qubits: Sequence[int], U, prec: int = SV_PREC_NATIVE) -> None:
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    m = _mat(U)
    _lib.check(_lib.load().sv_apply_fused(h, len(q), _iptr(q), _dptr(m), int(prec)))


def sv_probabilities(h, out=None) -> float:
    """Probabilities into ``out`` (CUDA float32/float64 tensor of 2^n, or
    None) and the FP64 total."""
    norm = ctypes.c_double()
    ptr = ctypes.c_void_p(out.data_ptr()) if out is not None else None
    _lib.check(_lib.load().sv_probabilities(h, ptr, ctypes.byref(norm)))
    return norm.value


def sv_expectation(h, z_masks: Sequence[int], coeffs: Sequence[float]) -> float:
    m = np.ascontiguousarray(z_masks, dtype=np.uint64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    out = ctypes.c_double()
    _lib.check(_lib.load().sv_expectation(h, len(m), _u64ptr(m), _dptr(c), ctypes.byref(out)))
    return out.value


def sv_expectation_noalloc(amps, n_qubits: int, z_masks: Sequence[int], coeffs: Sequence[float],
                           out, stream=None) -> None:
    """Expectation of a caller's state (CUDA complex64/complex128 tensor of
    2^n elements) written to ``out`` (a CUDA float64 tensor, element 0) on the
    stream, with no allocation and no host wait."""
    m = np.ascontiguousarray(z_masks, dtype=np.uint64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    s = stream if stream is not None else _current_stream()
    _lib.check(_lib.load().sv_expectation_noalloc(ctypes.c_void_p(amps.data_ptr()), int(n_qubits),
                                                 _dtype_code(amps.dtype), len(m), _u64ptr(m), _dptr(c),
                                                 ctypes.c_void_p(out.data_ptr()), s))


def sv_marginals(h, mask: int) -> np.ndarray:
    """FP64 outcome probabilities of the qubits of mask (at most 6)."""
    out = np.empty(1 << bin(mask).count("1"), np.float64)
    _lib.check(_lib.load().sv_marginals(h, mask, _dptr(out)))
    return out


def sv_collapse(h, mask: int, value: int) -> float:
    """Project onto (x & mask) == (value & mask) and renormalise; returns the probability."""
    p = ctypes.c_double()
    _lib.check(_lib.load().sv_collapse(h, mask, value, ctypes.byref(p)))
    return p.value


def sv_measure(h, mask: int, u: float) -> Tuple[int, float]:
    """Measure the qubits of mask with the uniform u in [0, 1); the state
    collapses.  Returns (outcome bits at the mask positions, probability)."""
    v = ctypes.c_uint64()
    p = ctypes.c_double()
    _lib.check(_lib.load().sv_measure(h, mask, u, ctypes.byref(v), ctypes.byref(p)))
    return int(v.value), p.value


def sv_sample(h, uniforms) -> np.ndarray:
    """Full-register outcomes for the given uniforms in [0, 1); state unchanged."""
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    out = np.empty(len(u), np.uint64)
    _lib.check(_lib.load().sv_sample(h, len(u), _dptr(u), _u64ptr(out)))
    return out


SV_OP_DTYPE = np.dtype([("kind", np.int32), ("n_targets", np.int32), ("targets", np.int32, (2,)),
                        ("ctrl_mask", np.uint64), ("param_index", np.int32), ("reserved", np.int32),
                        ("theta", np.float64), ("matrix", np.float64, (32,))])
assert SV_OP_DTYPE.itemsize == ctypes.sizeof(sv_op)


def ops_from_gates(gates) -> np.ndarray:
    """sv_op records (numpy structured array with the C layout) from symbolic
    gates (name, targets, controls, theta, param, matrix)."""
    n = len(gates)
    arr = np.zeros(max(1, n), dtype=SV_OP_DTYPE)
    if n == 0:
        return arr
    arr["kind"][:n] = [GATE_KINDS[g.name] for g in gates]
    arr["n_targets"][:n] = [len(g.targets) for g in gates]
    t = arr["targets"]
    t[:n, 0] = [g.targets[0] for g in gates]
    t[:n, 1] = [g.targets[1] if len(g.targets) > 1 else 0 for g in gates]
    arr["ctrl_mask"][:n] = [sum(1 << c for c in g.controls) for g in gates]
    arr["param_index"][:n] = [g.param for g in gates]
    arr["theta"][:n] = [g.theta for g in gates]
    for i, g in enumerate(gates):
        if g.name == "U":
            m = _mat(g.matrix)
            if m.size > 32:
                raise ValueError("sv_op holds at most a 4x4 matrix")
            arr["matrix"][i, :m.size] = m
    return arr


def _opptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.POINTER(sv_op))


def _params(params) -> tuple:
    if params is None:
        return None, 0, None
    p = np.ascontiguousarray(params, dtype=np.float64)
    return _dptr(p), len(p), p


def sv_run(h, gates, params=None, mode: int = SV_RUN_TILED) -> None:
    ops = ops_from_gates(gates)
    pp, n_p, keep = _params(params)
    _lib.check(_lib.load().sv_run(h, _opptr(ops), len(gates), pp, n_p, int(mode)))


def sv_schedule(n_qubits: int, dtype, gates, level: int = -1, params=None):
    """The passes of sv_run's tiled mode (host library, no GPU): (pass index
    of every gate as an int array, list of each pass's tile-qubit mask, 0 for
    a gate sv_run streams)."""
    ops = ops_from_gates(gates)
    pp, n_p, keep = _params(params)
    cap = max(1, len(gates))
    gp = np.full(max(1, len(gates)), -1, np.int32)
    pq = np.zeros(cap, np.uint64)
    npass = ctypes.c_int()
    _lib.check(_lib.load().sv_schedule(n_qubits, _dtype_code(dtype), _opptr(ops), len(gates), pp, n_p, int(level),
                                       cap, _iptr(gp), _u64ptr(pq), ctypes.byref(npass)))
    return gp[:len(gates)].copy(), [int(x) for x in pq[:npass.value]]


def sv_fuse(n_qubits: int, gates, k_max: int, params=None, max_blocks: Optional[int] = None):
    """Greedy fusion on the host library: list of (qubits, 2^k x 2^k matrix,
    number of gates absorbed)."""
    ops = ops_from_gates(gates)
    pp, n_p, keep = _params(params)
    cap = max_blocks or max(1, len(gates))
    bk = np.zeros(cap, np.int32)
    bq = np.full(cap * 5, -1, np.int32)
    bm = np.zeros(cap * 2 * 32 * 32, np.float64)
    bg = np.zeros(cap, np.int32)
    nb = ctypes.c_int()
    _lib.check(_lib.load().sv_fuse(n_qubits, _opptr(ops), len(gates), pp, n_p, k_max, cap, _iptr(bk),
                                   _iptr(bq), _dptr(bm), _iptr(bg), ctypes.byref(nb)))
    out = []
    for b in range(nb.value):
        k = int(bk[b])
        d = 1 << k
        m = bm[b * 2048:b * 2048 + 2 * d * d].view(np.complex128).reshape(d, d).copy()
        out.append((tuple(int(q) for q in bq[b * 5:b * 5 + k]), m, int(bg[b])))
    return out


def sv_run_fused(h, gates, k_max: int, prec: int, params=None) -> int:
    ops = ops_from_gates(gates)
    pp, n_p, keep = _params(params)
    nb = ctypes.c_int()
    _lib.check(_lib.load().sv_run_fused(h, _opptr(ops), len(gates), pp, n_p, int(k_max), int(prec),
                                        ctypes.byref(nb)))
    return nb.value


def sv_fused_tune(h, gates, k_max: int = 5, prec_mask: int = 0b111, reps: int = 1, params=None) -> dict:
    """Fastest of plain tile passes and fused passes (k in {4, 5} <= k_max,
    precisions in prec_mask) measured on the handle's state, which is left
    unchanged: {"k": 0 for plain, "prec": ..., "ms": ...}."""
    ops = ops_from_gates(gates)
    pp, n_p, keep = _params(params)
    k, p, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _lib.check(_lib.load().sv_fused_tune(h, _opptr(ops), len(gates), pp, n_p, int(k_max), int(prec_mask),
                                         int(reps), ctypes.byref(k), ctypes.byref(p), ctypes.byref(ms)))
    return {"k": k.value, "prec": p.value, "ms": ms.value}


def sv_adjoint_grad(h, lam, gates, params, z_masks, coeffs):
    ops = ops_from_gates(gates)
    p = np.ascontiguousarray(params, dtype=np.float64)
    m = np.ascontiguousarray(z_masks, dtype=np.uint64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    grad = np.zeros(len(p), np.float64)
    loss = ctypes.c_double()
    _lib.check(_lib.load().sv_adjoint_grad(h, lam, _opptr(ops), len(gates), _dptr(p), len(p), len(m),
                                           _u64ptr(m), _dptr(c), ctypes.byref(loss), _dptr(grad)))
    return loss.value, grad


# ------------------------------------------------------------------ Batch

class Batch:
    """Thousands of independent circuits run by one persistent kernel launch
    captured in a HIP graph (sv_batch_*).  ``circuits`` are objects with
    ``n`` and ``gates`` (parametrised gates must carry their angle in theta);
    the result of each circuit is <Z^{z_mask}>."""

    def __init__(self, circuits, dtype="c64", z_mask: int = 1, keep_states: bool = False,
                 stream=None):
        L = _lib.load()
        self.n = len(circuits)
        self.dtype = _dtype_code(dtype)
        self.widths = np.ascontiguousarray([c.n for c in circuits], dtype=np.int32)
        gates = [g for c in circuits for g in c.gates]
        offs = np.zeros(self.n + 1, dtype=np.int64)
        offs[1:] = np.cumsum([len(c.gates) for c in circuits])
        ops = ops_from_gates(gates)
        ops["param_index"] = -1  # angles are carried in theta
        h = ctypes.c_void_p()
        s = stream if stream is not None else _current_stream()
        _lib.check(L.sv_batch_create(self.n, _iptr(self.widths),
                                     offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _opptr(ops), None, 0,
                                     self.dtype, int(z_mask), _lib.SV_BATCH_KEEP_STATES if keep_states else 0,
                                     s, ctypes.byref(h)))
        self.handle = h

    def run(self) -> "Batch":
        _lib.check(_lib.load().sv_batch_run(self.handle))
        return self

    def results(self) -> np.ndarray:
        out = np.zeros(self.n, np.float64)
        _lib.check(_lib.load().sv_batch_results(self.handle, _dptr(out)))
        return out

    def state(self, i: int) -> np.ndarray:
        dt = np.complex64 if self.dtype == SV_C64 else np.complex128
        out = np.zeros(1 << int(self.widths[i]), dt)
        _lib.check(_lib.load().sv_batch_state(self.handle, int(i), ctypes.c_void_p(out.ctypes.data)))
        return out

    def tune(self, reps: int = 2):
        m, w, g, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        t = ctypes.c_double()
        _lib.check(_lib.load().sv_batch_tune(self.handle, int(reps), ctypes.byref(m), ctypes.byref(w),
                                             ctypes.byref(g), ctypes.byref(f), ctypes.byref(t)))
        return {"tile_qubits": m.value, "sweep_width": w.value, "grid": g.value, "fuse_width": f.value,
                "ms": t.value}

    def config(self, tile_qubits: int, sweep_width: int, grid: int, fuse_width: int = 0) -> "Batch":
        """Rebuild the program and graph for one launch configuration."""
        _lib.check(_lib.load().sv_batch_config(self.handle, int(tile_qubits), int(sweep_width), int(grid),
                                               int(fuse_width)))
        return self

    def close(self):
        if getattr(self, "handle", None) is not None:
            _lib.check(_lib.load().sv_batch_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ State

class _Op:
    """A queued gate in the form ops_from_gates reads."""

    __slots__ = ("name", "targets", "controls", "theta", "param", "matrix")

    def __init__(self, name, targets, controls=(), theta=0.0, matrix=None):
        self.name = name
        self.targets = tuple(int(q) for q in targets)
        self.controls = tuple(int(q) for q in controls)
        self.theta = float(theta)
        self.param = -1
        self.matrix = matrix


class State:
    """An n-qubit register whose amplitudes live in a torch CUDA tensor.

    Besides the entry-point wrappers it offers the register interface of the
    paper's library (Sec. 2.3 gates, App. B/C usage): gate methods ``h``,
    ``x``, ``y``, ``z``, ``s``, ``t``, ``rx``, ``ry``, ``rz``, ``u1``,
    ``cx``, ``cz``, ``cu1`` and ``apply_gate`` queue the gate, as the
    paper's kernels are queued on a device command queue, and every read of
    the register (probabilities, amplitudes, measurement, ``sync``) first
    runs the queued gates in one ``sv_run`` (tile-pass schedule), so
    consecutive gates share trips of the state through HBM.
    ``measure(samples=k)`` returns the outcome counts as in App. C."""

    def __init__(self, n_qubits: int, dtype="c128", device=None):
        torch = _torch()
        code = _dtype_code(dtype)
        self.n = n_qubits
        self.dtype = code
        self._pending = []
        tdt = torch.complex64 if code == SV_C64 else torch.complex128
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(dev):
            self.amps = torch.empty(1 << n_qubits, dtype=tdt, device=dev)
            self.handle = sv_alloc(n_qubits, code, self.amps, _current_stream())
        self.device = dev

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            sv_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------- queued gates
    def _queue(self, name, targets, controls=(), theta=0.0, matrix=None) -> "State":
        for q in tuple(targets) + tuple(controls):
            if not 0 <= int(q) < self.n:
                raise ValueError(f"qubit {q} outside the {self.n}-qubit register")
        self._pending.append(_Op(name, targets, controls, theta, matrix))
        return self

    def flush(self) -> "State":
        """Run the queued gates (one sv_run, tile-pass schedule)."""
        if self._pending:
            ops, self._pending = self._pending, []
            sv_run(self.handle, ops, None, SV_RUN_TILED)
        return self

    def h(self, target: int) -> "State":
        return self._queue("H", (target,))

    def x(self, target: int) -> "State":
        return self._queue("X", (target,))

    def y(self, target: int) -> "State":
        return self._queue("Y", (target,))

    def z(self, target: int) -> "State":
        return self._queue("Z", (target,))

    def s(self, target: int) -> "State":
        return self._queue("S", (target,))

    def t(self, target: int) -> "State":
        return self._queue("T", (target,))

    def rx(self, target: int, theta: float) -> "State":
        return self._queue("RX", (target,), (), theta)

    def ry(self, target: int, theta: float) -> "State":
        return self._queue("RY", (target,), (), theta)

    def rz(self, target: int, theta: float) -> "State":
        return self._queue("RZ", (target,), (), theta)

    def u1(self, target: int, theta: float) -> "State":
        return self._queue("U1", (target,), (), theta)

    def cx(self, control: int, target: int) -> "State":
        return self._queue("X", (target,), (control,))

    def cz(self, control: int, target: int) -> "State":
        return self._queue("Z", (target,), (control,))

    def cu1(self, control: int, target: int, theta: float) -> "State":
        """diag(1, 1, 1, e^{i theta}) on (control, target) (symmetric)."""
        return self._queue("U1", (target,), (control,), theta)

    def apply_gate(self, U, target, controls: Iterable[int] = ()) -> "State":
        """A 2x2 (one target) or 4x4 (two targets, bit j of the matrix index
        = targets[j]) unitary, optionally controlled."""
        targets = (target,) if np.isscalar(target) else tuple(target)
        return self._queue("U", targets, tuple(controls), 0.0, np.asarray(U, dtype=np.complex128))

    # ----------------------------------------------------- entry points
    def set_basis(self, x: int) -> "State":
        self._pending = []
        sv_set_basis(self.handle, x)
        return self

    def apply(self, U, targets, controls: Iterable[int] = ()) -> "State":
        self.flush()
        mask = 0
        for c in controls:
            mask |= 1 << c
        sv_apply_gate(self.handle, list(targets), U, mask)
        return self

    def apply_fused(self, U, qubits, prec: int = SV_PREC_NATIVE) -> "State":
        self.flush()
        sv_apply_fused(self.handle, list(qubits), U, prec)
        return self

    def run(self, gates, params=None, mode: int = SV_RUN_TILED) -> "State":
        self.flush()
        sv_run(self.handle, gates, params, mode)
        return self

    def run_fused(self, gates, k_max: int = 5, prec: int = SV_PREC_FP32, params=None) -> int:
        self.flush()
        return sv_run_fused(self.handle, gates, k_max, prec, params)

    def fused_tune(self, gates, k_max: int = 5, prec_mask: int = 0b111, reps: int = 1, params=None) -> dict:
        self.flush()
        return sv_fused_tune(self.handle, gates, k_max, prec_mask, reps, params)

    def probabilities(self, out=None) -> float:
        self.flush()
        return sv_probabilities(self.handle, out)

    def expectation(self, z_masks, coeffs) -> float:
        self.flush()
        return sv_expectation(self.handle, z_masks, coeffs)

    def marginals(self, mask: int) -> np.ndarray:
        self.flush()
        return sv_marginals(self.handle, mask)

    def collapse(self, mask: int, value: int) -> float:
        self.flush()
        return sv_collapse(self.handle, mask, value)

    def measure(self, mask: Optional[int] = None, u: Optional[float] = None, *, samples: Optional[int] = None,
                seed: int = 0):
        """``measure(mask, u)``: measure the qubits of ``mask`` with the
        uniform ``u`` (outcome, probability; the register collapses).
        ``measure(samples=k)``: k samples of all qubits drawn from the
        register without changing it, returned as counts keyed by the
        outcome's bit string (qubit n-1 first); the uniforms come from
        numpy's generator seeded with ``seed``."""
        self.flush()
        if samples is not None:
            if mask is not None or u is not None:
                raise ValueError("measure takes either (mask, u) or samples")
            uniforms = np.random.default_rng(seed).random(int(samples))
            counts = {}
            for x in sv_sample(self.handle, uniforms):
                key = format(int(x), f"0{self.n}b")
                counts[key] = counts.get(key, 0) + 1
            return counts
        if mask is None or u is None:
            raise ValueError("measure takes either (mask, u) or samples")
        return sv_measure(self.handle, mask, u)

    def sample(self, uniforms) -> np.ndarray:
        self.flush()
        return sv_sample(self.handle, uniforms)

    def sync(self) -> "State":
        self.flush()
        sv_sync(self.handle)
        return self

    def numpy(self) -> np.ndarray:
        self.sync()
        return self.amps.cpu().numpy()
