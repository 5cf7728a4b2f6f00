"""GPU parity of dense fused blocks (native, FP32 MFMA, split-BF16 MFMA)
against the FP64 oracle.

Tolerances.  A block output is a 2^k-term sum; in FP32 its rounding error
is at most 2^k * 4 eps32 times the group's norm, so a normalised state moves
by at most that in 2-norm per block.  Split-BF16 represents each FP32
operand as hi + lo with relative error <= 2^-17 per operand and drops the
lo*lo product (<= 2^-18), so each product is within 2^-15 relative and a
block output within 2^k * 2^-15 of the group norm.  A pass that the cost
model runs as plain register sweeps rounds like sv_run (4 sqrt(2) eps32
per gate), so gate lists add that bound for all their gates.  Every run
also checks the fidelity target 1 - F <= 1e-6; complex128 blocks are held
to 1e-12."""

import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from helpers import C128_ATOL, EPS32, c64_bound, fidelity, random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1805_00988_amd as sv  # noqa: E402

O.build(force=False)

NP_DT = {"c128": np.complex128, "c64": np.complex64}
PRECS = {"native": sv.SV_PREC_NATIVE, "fp32": sv.SV_PREC_FP32, "bf16x3": sv.SV_PREC_SPLIT_BF16}


def block_bound(k, prec, n_blocks=1):
    per = (2 ** k) * (4 * EPS32 if prec in ("native", "fp32") else 2.0 ** -15)
    return per * n_blocks


def check(got, ref, dtype, prec, k, n_blocks=1, n_gates=0):
    got = got.astype(np.complex128)
    err = float(np.max(np.abs(got - ref)))
    if dtype == "c128":
        assert err <= C128_ATOL, err
    else:
        bound = block_bound(k, prec, n_blocks) + (c64_bound(n_gates) if n_gates else 0.0)
        assert err <= bound, (err, bound)
        assert 1.0 - fidelity(got, ref) <= 1e-6
    return err


def start(n, dtype, seed):
    psi0 = random_state(n, seed)
    st = sv.State(n, dtype)
    st.amps.copy_(torch.from_numpy(psi0.astype(NP_DT[dtype])))
    return st, psi0.astype(NP_DT[dtype]).astype(np.complex128)


@pytest.mark.parametrize("dtype,prec", [("c128", "native"), ("c64", "native"), ("c64", "fp32"),
                                        ("c64", "bf16x3")])
@pytest.mark.parametrize("n", [10, 14, 17])
def test_single_block_random_unitary(dtype, prec, n):
    rng = np.random.default_rng(n)
    ks = [1, 2, 3, 4, 5] if prec == "native" else [4, 5]
    qubit_sets = []
    for k in ks:
        qubit_sets.append(list(range(k)))                              # lowest qubits
        qubit_sets.append(list(range(n - k, n)))                       # highest
        qubit_sets.append([int(q) for q in rng.choice(n, size=k, replace=False)])  # scattered, unsorted
    for i, qs in enumerate(qubit_sets):
        k = len(qs)
        U = C.random_unitary(1 << k, rng)
        st, psi = start(n, dtype, seed=i)
        st.apply_fused(U, qs, PRECS[prec])
        O.apply_kq(psi, n, qs, U)
        check(st.numpy(), psi, dtype, prec, k)


@pytest.mark.parametrize("dtype,prec", [("c128", "native"), ("c64", "native"), ("c64", "fp32"),
                                        ("c64", "bf16x3")])
@pytest.mark.parametrize("k", [4, 5])
@pytest.mark.parametrize("n", [12, 16, 18])
def test_run_fused_config2_recipe(dtype, prec, k, n):
    """Config-2 recipe (1q layer + CZ on random pairs) at reduced size."""
    circ = C.config2(n=n, seed=n + k, depth=12)
    st = sv.State(n, dtype)
    nb = st.run_fused(circ.gates, k_max=k, prec=PRECS[prec])
    assert 0 <= nb < len(circ.gates)
    check(st.numpy(), O.run(circ), dtype, prec, k, nb, len(circ.gates))


@pytest.mark.parametrize("dtype,prec", [("c128", "native"), ("c64", "fp32"), ("c64", "bf16x3")])
def test_run_fused_qft_and_cnot_circuits(dtype, prec):
    for circ in (C.qft_circuit(15, 12345), C.random_circuit(15, 10, 3, "X"), C.config0(1)):
        st = sv.State(circ.n, dtype).set_basis(circ.basis)
        nb = st.run_fused(circ.gates, k_max=5, prec=PRECS[prec])
        check(st.numpy(), O.run(circ), dtype, prec, 5, nb, len(circ.gates))


def diagonal_rich_circuit(n, seed, layers=6):
    """Dense one-qubit layers interleaved with diagonal gates of 1-5 qubits
    (controlled phases, controlled RZ, two-qubit diagonal matrices with
    controls), whose qubits are spread over the whole register so that many
    of them lie outside a fused pass's tile."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            gates.append(C.Gate(str(rng.choice(["H", "RX", "RY"])), (q,), theta=float(rng.uniform(0, 2 * math.pi))))
        for _ in range(n):
            w = int(rng.integers(1, 6))
            qs = [int(x) for x in rng.choice(n, size=w, replace=False)]
            kind = int(rng.integers(0, 3))
            th = float(rng.uniform(0, 2 * math.pi))
            if kind == 2 and w >= 2:
                ph = np.exp(1j * rng.uniform(0, 2 * math.pi, size=4))
                gates.append(C.Gate("U", (qs[0], qs[1]), tuple(qs[2:]), matrix=np.diag(ph)))
            else:
                gates.append(C.Gate("U1" if kind == 0 else "RZ", (qs[0],), tuple(qs[1:]), theta=th))
    return C.Circuit(n, gates, 0, None, f"diag_rich_n{n}_s{seed}")


@pytest.mark.parametrize("dtype,prec", [("c128", "native"), ("c64", "native"), ("c64", "fp32"),
                                        ("c64", "bf16x3")])
@pytest.mark.parametrize("n", [15, 17])
def test_run_fused_diagonal_gates_outside_tile(dtype, prec, n):
    """Diagonal gates may keep qubits outside a fused pass's tile (their
    blocks then carry one matrix per value of those qubits); the result must
    still match the oracle."""
    circ = diagonal_rich_circuit(n, 40 + n)
    st, psi0 = start(n, dtype, 60 + n)
    nb = st.run_fused(circ.gates, k_max=5, prec=PRECS[prec])
    check(st.numpy(), O.run_gates(n, circ.gates, psi0), dtype, prec, 5, nb, len(circ.gates))


@pytest.mark.parametrize("dtype,prec", [("c128", "native"), ("c64", "bf16x3")])
def test_run_fused_only_outside_diagonals(dtype, prec):
    """A pass whose gates act only on qubits outside the tile: its blocks have
    no qubit of their own (a phase per tile), padded to the pass's width."""
    n = 18
    gates = [C.Gate("Z", (17,), (16,)), C.Gate("U1", (15,), (17,), theta=0.7),
             C.Gate("RZ", (16,), theta=1.3), C.Gate("T", (14,)), C.Gate("S", (17,), (14, 15, 16))]
    st, psi0 = start(n, dtype, 7)
    nb = st.run_fused(gates, k_max=4, prec=PRECS[prec])
    check(st.numpy(), O.run_gates(n, gates, psi0), dtype, prec, 4, nb, len(gates))


def test_mfma_rejected_for_complex128():
    st = sv.State(12, "c128")
    with pytest.raises(sv.SVError):
        st.apply_fused(np.eye(16), [0, 1, 2, 3], sv.SV_PREC_FP32)


def kernel_launches(st):
    """Launches per kernel kind recorded since timing was switched on."""
    import ctypes
    from paper_1805_00988_amd import _lib
    lib = _lib.load()
    arr = (_lib.sv_kernel_stat * 16)()
    n = ctypes.c_int()
    _lib.check(lib.sv_timing_read(st.handle, arr, 16, ctypes.byref(n)))
    return {arr[i].name.decode(): int(arr[i].launches) for i in range(n.value)}


@pytest.mark.parametrize("dtype,prec", [("c128", "native"), ("c64", "bf16x3")])
def test_run_fused_passes_chosen_plain(dtype, prec):
    """A QFT (phase gates and Hadamards) through sv_run_fused: the cost model
    runs its passes as plain register sweeps (tile-pass launches, no dense
    blocks), matching the closed form and the oracle."""
    from paper_1805_00988_amd import _lib
    circ = C.qft_circuit(17, 12345)
    st = sv.State(17, dtype).set_basis(circ.basis)
    _lib.check(_lib.load().sv_timing(st.handle, 1))
    nb = st.run_fused(circ.gates, k_max=5, prec=PRECS[prec])
    runs = kernel_launches(st)
    assert runs.get("tile_pass", 0) > 0 and nb == 0, (runs, nb)
    check(st.numpy(), O.run(circ), dtype, prec, 5, nb, len(circ.gates))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_fused_tune_keeps_state_and_choice_matches_oracle(dtype):
    """sv_fused_tune measures plain and fused candidates from the handle's
    state, leaves that state bit for bit unchanged, and its choice applied to
    the same state matches the oracle."""
    n = 16
    circ = C.config2(n=n, seed=20, depth=12)
    st, psi0 = start(n, dtype, 21)
    before = st.numpy().copy()
    choice = st.fused_tune(circ.gates, k_max=5, prec_mask=0b111, reps=1)
    np.testing.assert_array_equal(st.numpy(), before)
    assert choice["k"] in (0, 4, 5) and choice["ms"] > 0.0
    if dtype == "c128":
        assert choice["prec"] == sv.SV_PREC_NATIVE
    ref = O.run_gates(n, circ.gates, psi0)
    if choice["k"] == 0:
        st.run(circ.gates, mode=sv.SV_RUN_TILED)
        check(st.numpy(), ref, dtype, "native", 4, 0, len(circ.gates))
    else:
        nb = st.run_fused(circ.gates, k_max=choice["k"], prec=choice["prec"])
        pname = {v: k for k, v in PRECS.items()}[choice["prec"]]
        check(st.numpy(), ref, dtype, pname, choice["k"], nb, len(circ.gates))
