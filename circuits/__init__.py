"""Seeded synthetic circuit generators.

This module is the only code shared by the FP64 oracle and the HIP path: it
draws random circuits and emits them as symbolic gate lists (gate name, target
qubits, control qubits, angle, parameter index).  It holds none of the
simulation arithmetic: gate matrices, amplitude updates, probabilities and
expectations are computed independently by each side from the gate names.

Conventions (the paper's kernels and its Bernstein-Vazirani example index the
state with qubit q as bit q of the amplitude index):

* qubit q is bit q of the basis-state index (qubit 0 is the least significant);
* a gate with ``controls`` acts only on the subspace where every control bit
  is 1 (the controlled variant of the gate-application algorithm, Sec. 2.3);
* for a multi-qubit gate, bit j of the local row/column index of its matrix is
  the value of qubit ``targets[j]``.

Gate names: H X Y Z S T (fixed one-qubit gates), RX RY RZ (rotations
exp(-i theta P / 2)), U1 (phase diag(1, e^{i theta})), U (an explicit unitary
carried in ``matrix``, 2^k x 2^k complex).  CNOT, CZ and CU1 are X, Z and U1
with one control.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

FIXED_1Q = ("H", "X", "Y", "Z", "S", "T")
ROT_1Q = ("RX", "RY", "RZ")
RANDOM_1Q_SET = FIXED_1Q + ROT_1Q          # the one-qubit gate menu of the random circuits
PARAM_NAMES = ("RX", "RY", "RZ", "U1")


@dataclass(frozen=True)
class Gate:
    name: str
    targets: Tuple[int, ...]
    controls: Tuple[int, ...] = ()
    theta: float = 0.0
    param: int = -1                      # index into a parameter vector, -1 = fixed angle
    matrix: Optional[np.ndarray] = field(default=None, compare=False)

    @property
    def qubits(self) -> Tuple[int, ...]:
        return tuple(self.targets) + tuple(self.controls)


@dataclass
class Circuit:
    n: int
    gates: List[Gate]
    basis: int = 0                       # initial basis state |basis>
    params: Optional[np.ndarray] = None  # parameter vector for gates with param >= 0
    name: str = ""

    def __len__(self) -> int:
        return len(self.gates)

    def updates(self) -> int:
        """Gate-amplitude updates: 2^n per gate, halved per control qubit."""
        return sum((1 << self.n) >> len(g.controls) for g in self.gates)

    def bound(self) -> "Circuit":
        """Copy whose parametrised gates carry theta = params[param]."""
        if self.params is None:
            return self
        gs = [Gate(g.name, g.targets, g.controls,
                   float(self.params[g.param]) if g.param >= 0 else g.theta,
                   g.param, g.matrix) for g in self.gates]
        return Circuit(self.n, gs, self.basis, self.params, self.name)


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _random_layer_1q(rng: np.random.Generator, n: int) -> List[Gate]:
    gates = []
    for q in range(n):
        name = RANDOM_1Q_SET[int(rng.integers(len(RANDOM_1Q_SET)))]
        theta = float(rng.uniform(0.0, 2.0 * math.pi))
        gates.append(Gate(name, (q,), (), theta if name in ROT_1Q else 0.0))
    return gates


def _random_pairs(rng: np.random.Generator, n: int, count: int) -> List[Tuple[int, int]]:
    perm = rng.permutation(n)
    return [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(count)]


def random_circuit(n: int, depth: int, seed: int, entangler: str = "X",
                   pairs_per_layer: Optional[int] = None) -> Circuit:
    """Layers of one random one-qubit gate per qubit followed by controlled
    entanglers (CNOT for ``entangler='X'``, CZ for ``'Z'``) on disjoint random
    qubit pairs; the first qubit of each pair is the control."""
    rng = _rng(seed)
    if pairs_per_layer is None:
        pairs_per_layer = n // 2
    gates: List[Gate] = []
    for _ in range(depth):
        gates += _random_layer_1q(rng, n)
        for c, t in _random_pairs(rng, n, pairs_per_layer):
            gates.append(Gate(entangler, (t,), (c,)))
    return Circuit(n, gates, 0, None, f"random_n{n}_d{depth}_s{seed}")


def qft_circuit(n: int, basis: int = 0) -> Circuit:
    """The QFT circuit of the paper's benchmark: for each qubit j, controlled
    phases of pi/2^(j-k) between j and every lower qubit k, then H on j; no
    final swaps.  The controlled phase is symmetric, qubit j is the control."""
    gates: List[Gate] = []
    for j in range(n):
        for k in range(j):
            gates.append(Gate("U1", (k,), (j,), math.pi / float(2 ** (j - k))))
        gates.append(Gate("H", (j,)))
    return Circuit(n, gates, basis, None, f"qft_n{n}_x{basis}")


def random_basis(n: int, seed: int) -> int:
    return int(_rng(seed).integers(0, 1 << n, dtype=np.uint64))


def qft_random_basis(n: int, seed: int) -> Circuit:
    return qft_circuit(n, random_basis(n, seed))


def hea_circuit(n: int, layers: int, seed: int, entangler: str = "ladder",
                params: Optional[np.ndarray] = None) -> Circuit:
    """Hardware-efficient ansatz: per layer RY then RZ on every qubit, then a
    CNOT ladder (q -> q+1) or ring (q -> (q+1) mod n).  Parameter index of the
    rotation on qubit q in layer l is (l*n + q)*2 + (0 for RY, 1 for RZ)."""
    n_params = layers * n * 2
    if params is None:
        params = _rng(seed).uniform(0.0, 2.0 * math.pi, size=n_params)
    params = np.asarray(params, dtype=np.float64)
    gates: List[Gate] = []
    for l in range(layers):
        for q in range(n):
            p = (l * n + q) * 2
            gates.append(Gate("RY", (q,), (), float(params[p]), p))
            gates.append(Gate("RZ", (q,), (), float(params[p + 1]), p + 1))
        if entangler == "ladder":
            pairs = [(q, q + 1) for q in range(n - 1)]
        elif entangler == "ring":
            pairs = [(q, (q + 1) % n) for q in range(n)] if n > 2 else [(0, 1)]
        else:
            raise ValueError(entangler)
        for c, t in pairs:
            gates.append(Gate("X", (t,), (c,)))
    return Circuit(n, gates, 0, params, f"hea_{entangler}_n{n}_l{layers}_s{seed}")


def zz_ring_observable(n: int) -> Tuple[List[int], List[float]]:
    """Sum_i Z_i Z_{(i+1) mod n} as (Z-masks, coefficients)."""
    masks = [(1 << i) | (1 << ((i + 1) % n)) for i in range(n)]
    return masks, [1.0] * n


def random_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary from the QR decomposition of a complex Gaussian."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def random_unitary_gates(n: int, count: int, k: int, seed: int, max_controls: int = 0) -> Circuit:
    """Explicit random k-qubit unitaries on random distinct qubits, each with
    up to ``max_controls`` random control qubits."""
    rng = _rng(seed)
    gates = []
    for _ in range(count):
        qs = [int(v) for v in rng.choice(n, size=min(n, k + max_controls), replace=False)]
        nc = int(rng.integers(0, max_controls + 1)) if max_controls else 0
        gates.append(Gate("U", tuple(qs[:k]), tuple(qs[k:k + nc]), 0.0, -1,
                          random_unitary(1 << k, rng)))
    return Circuit(n, gates, 0, None, f"unitary{k}_n{n}_c{count}_s{seed}")


def batch_hea(count: int, wmin: int, wmax: int, layers: int, seed: int) -> List[Circuit]:
    """``count`` independent ladder-HEA circuits of widths uniform in
    [wmin, wmax], each with its own angles."""
    rng = _rng(seed)
    widths = rng.integers(wmin, wmax + 1, size=count)
    out = []
    for i, w in enumerate(widths):
        params = rng.uniform(0.0, 2.0 * math.pi, size=layers * int(w) * 2)
        c = hea_circuit(int(w), layers, 0, "ladder", params)
        c.name = f"batch{i}_w{int(w)}"
        out.append(c)
    return out


# --- the five workload recipes -------------------------------------------------

def config0(seed: int = 0) -> Circuit:
    """12 qubits from |0>, depth 20: one random one-qubit gate per qubit, then
    CNOTs on 6 random disjoint pairs, per layer (complex128)."""
    return random_circuit(12, 20, seed, "X", 6)


def config1(n: int, seed: int = 0) -> List[Circuit]:
    """Plain path at scale: QFT on a seeded random basis state, then a depth-20
    random circuit with n//2 CNOTs per layer."""
    return [qft_random_basis(n, seed), random_circuit(n, 20, seed + 1000, "X", n // 2)]


def config2(n: int = 30, seed: int = 0, depth: int = 40) -> Circuit:
    """Fusion workload: depth-40 random layers of one-qubit gates plus CZ on
    n//2 random disjoint pairs."""
    return random_circuit(n, depth, seed, "Z", n // 2)


def config3(seed: int = 0, count: int = 4096, wmin: int = 10, wmax: int = 20,
            layers: int = 8) -> List[Circuit]:
    return batch_hea(count, wmin, wmax, layers, seed)


def config4(seed: int = 0, n: int = 24, layers: int = 12) -> Tuple[Circuit, List[int], List[float]]:
    c = hea_circuit(n, layers, seed, "ring")
    masks, coeffs = zz_ring_observable(n)
    return c, masks, coeffs


def bernstein_vazirani(n: int, a: int) -> Circuit:
    """H on every qubit, Z on the set bits of a (inner-product oracle), H on
    every qubit (App. C)."""
    gates = [Gate("H", (q,)) for q in range(n)]
    gates += [Gate("Z", (q,)) for q in range(n) if (a >> q) & 1]
    gates += [Gate("H", (q,)) for q in range(n)]
    return Circuit(n, gates, 0, None, f"bv_n{n}_a{a}")


def block_product_circuit(n: int, block: int, depth: int, seed: int) -> Tuple[Circuit, List[List[int]]]:
    """A random circuit whose entanglers stay inside fixed qubit blocks (a
    random partition of the n qubits into blocks of ``block`` qubits, the last
    one ragged).  The final state is the tensor product of the block states, so
    any single amplitude of an n-qubit run can be checked from small block
    simulations.  Returns the circuit and the qubit lists of the blocks."""
    rng = _rng(seed)
    perm = [int(v) for v in rng.permutation(n)]
    blocks = [sorted(perm[i:i + block]) for i in range(0, n, block)]
    gates: List[Gate] = []
    for _ in range(depth):
        gates += _random_layer_1q(rng, n)
        for b in blocks:
            if len(b) < 2:
                continue
            sub = [b[int(i)] for i in rng.permutation(len(b))]
            for i in range(len(b) // 2):
                gates.append(Gate("X" if rng.integers(2) else "Z", (sub[2 * i + 1],), (sub[2 * i],)))
    return Circuit(n, gates, 0, None, f"blocks_n{n}_b{block}_d{depth}_s{seed}"), blocks


def uniforms(count: int, seed: int) -> np.ndarray:
    """Seeded uniforms in [0, 1): the random draws of measurement and sampling
    are inputs to both the oracle and the library."""
    return _rng(seed).random(count)
