"""The host greedy fuser (sv_fuse, no GPU needed) against the FP64 oracle.

Pin: applying the fused blocks with the oracle's own k-qubit loop in FP64
reproduces the unfused oracle run, so the blocks are exactly the product of
the gates they absorb, in an order that respects every shared qubit."""

import numpy as np
import pytest

import circuits as C
import oracle as O
import paper_1805_00988_amd as sv

O.build(force=False)


def apply_blocks(n, blocks, psi):
    for qubits, M, _ in blocks:
        O.apply_kq(psi, n, list(qubits), M)
    return psi


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("maker", ["config0", "cz", "qft", "unitary2", "hea"])
def test_fused_blocks_reproduce_circuit(k, maker):
    if maker == "config0":
        circ = C.random_circuit(9, 8, 1, "X", 4)
    elif maker == "cz":
        circ = C.config2(n=10, seed=2, depth=6)
    elif maker == "qft":
        circ = C.qft_circuit(9, 311)
    elif maker == "unitary2":
        circ = C.random_unitary_gates(8, 20, 2, seed=5, max_controls=1)
    else:
        circ = C.hea_circuit(8, 3, 4, "ring")
    if any(len(g.qubits) > k for g in circ.gates):
        with pytest.raises(sv.SVError):
            sv.sv_fuse(circ.n, circ.gates, k, params=circ.params)
        return
    blocks = sv.sv_fuse(circ.n, circ.gates, k, params=circ.params)
    assert sum(b[2] for b in blocks) == len(circ.gates)
    assert all(1 <= len(b[0]) <= k for b in blocks)
    assert all(list(b[0]) == sorted(b[0]) for b in blocks)
    if k >= 3:
        assert len(blocks) < len(circ.gates)
    for qubits, M, _ in blocks:
        np.testing.assert_allclose(M.conj().T @ M, np.eye(M.shape[0]), atol=1e-12)
    ref = O.run(circ)
    got = apply_blocks(circ.n, blocks, O.basis_state(circ.n, circ.basis))
    np.testing.assert_allclose(got, ref, atol=1e-12, rtol=0)


def test_fusion_absorbs_whole_config2_layers():
    circ = C.config2(n=30, seed=0, depth=40)
    b4 = sv.sv_fuse(circ.n, circ.gates, 4)
    b5 = sv.sv_fuse(circ.n, circ.gates, 5)
    assert sum(b[2] for b in b5) == len(circ.gates) == 1800
    assert len(b5) < len(b4) < len(circ.gates)


def test_fuse_rejects_bad_arguments():
    circ = C.random_circuit(5, 2, 0)
    with pytest.raises(sv.SVError):
        sv.sv_fuse(5, circ.gates, 0)
    with pytest.raises(sv.SVError):
        sv.sv_fuse(5, circ.gates, 6)
    with pytest.raises(sv.SVError):
        sv.sv_fuse(4, circ.gates, 3)  # qubit 4 outside a 4-qubit register
