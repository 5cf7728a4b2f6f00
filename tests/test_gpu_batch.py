"""GPU parity of the batched persistent kernel (sv_batch_*) against the
FP64 oracle: final states (kept for inspection) and Z-string expectations
per circuit, repeated graph replays, the autotuner, and the full batched
workload (4096 ladder-ansatz circuits of 10..20 qubits) on a sampled subset."""

import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from helpers import C128_ATOL, c64_bound, fidelity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1805_00988_amd as sv  # noqa: E402

O.build(force=False)


def mixed_circuits(dtype, count, seed):
    rng = np.random.default_rng(seed)
    wmin = 4 if dtype == "c64" else 3
    out = []
    for i in range(count):
        w = int(rng.integers(wmin, 17))
        kind = i % 3
        if kind == 0:
            c = C.hea_circuit(w, 3, seed=i, entangler="ladder").bound()
        elif kind == 1:
            c = C.random_circuit(w, 4, seed=i, entangler="X")
        else:
            c = C.config2(n=w, seed=i, depth=3)
        out.append(c)
    return out


def z_of(psi, n, zmask):
    return O.expectation_z(psi, n, [zmask], [1.0])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batch_states_and_expectations(dtype):
    circs = mixed_circuits(dtype, 40, seed=1)
    b = sv.Batch(circs, dtype, z_mask=1, keep_states=True)
    first = None
    for rep in range(3):
        b.run()
        z = b.results()
        # eager work on the same stream between replays
        x = torch.ones(1024, device="cuda")
        torch.cuda.synchronize()
        assert float(x.sum()) == 1024.0
        if first is None:
            first = z.copy()
        np.testing.assert_array_equal(z, first)
    for i, c in enumerate(circs):
        ref = O.run(c)
        got = b.state(i).astype(np.complex128)
        err = np.max(np.abs(got - ref))
        if dtype == "c128":
            assert err <= C128_ATOL, (i, c.n, err)
            assert abs(first[i] - z_of(ref, c.n, 1)) <= 1e-12
        else:
            assert err <= c64_bound(len(c)), (i, c.n, err)
            assert 1.0 - fidelity(got, ref) <= 1e-6
            assert abs(first[i] - z_of(ref, c.n, 1)) <= 2 * c64_bound(len(c))
    b.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batch_gateless_and_diagonal_circuits(dtype):
    """Circuits without gates (|0...0>, <Z_0> = 1) and circuits of phase
    gates only, one tile wide and wider than a tile, mixed with ordinary
    ones: the first sweep synthesises |0...0> in registers and the last
    reduces from registers."""
    circs = []
    for w in (5, 13, 15):
        circs.append(C.Circuit(w, [], 0, None, f"empty_{w}"))
        gates = [C.Gate("H", (q,)) for q in range(w)]
        gates += [C.Gate("U1", (q,), ((q + 1) % w,), 0.3 + 0.1 * q) for q in range(w)]
        gates += [C.Gate("Z", (q,)) for q in range(0, w, 2)]
        circs.append(C.Circuit(w, gates, 0, None, f"phases_{w}"))
    circs += mixed_circuits(dtype, 6, seed=7)
    b = sv.Batch(circs, dtype, z_mask=1, keep_states=True)
    b.run()
    z = b.results()
    for i, c in enumerate(circs):
        ref = O.run(c)
        got = b.state(i).astype(np.complex128)
        tol = C128_ATOL if dtype == "c128" else c64_bound(max(1, len(c)))
        assert np.max(np.abs(got - ref)) <= tol, (i, c.n)
        assert abs(z[i] - z_of(ref, c.n, 1)) <= 2 * tol, (i, c.n)
    b.close()


def test_batch_autotuner_keeps_results():
    circs = mixed_circuits("c64", 64, seed=2)
    b = sv.Batch(circs, "c64", z_mask=0b101)
    b.run()
    before = b.results()
    choice = b.tune(reps=1)
    assert choice["tile_qubits"] in (11, 12, 13) and choice["sweep_width"] in (3, 4)
    assert choice["fuse_width"] in (0, 1, 2)
    b.run()
    after = b.results()
    for i, c in enumerate(circs):
        ref = z_of(O.run(c), c.n, 0b101)
        assert abs(before[i] - ref) <= 2 * c64_bound(len(c))
        assert abs(after[i] - ref) <= 2 * c64_bound(len(c))
    b.close()


def test_batch_autotuner_complex128_narrow_circuits():
    """The tuner's sweep-width candidates never exceed the narrowest circuit:
    a complex128 batch holding 3-qubit circuits keeps correct results for
    whatever (tile, sweep width, grid) it picks."""
    rng = np.random.default_rng(11)
    circs = [C.hea_circuit(3, 3, seed=i, entangler="ladder").bound() for i in range(6)]
    circs += [C.random_circuit(int(rng.integers(3, 15)), 4, seed=50 + i, entangler="X") for i in range(18)]
    b = sv.Batch(circs, "c128", z_mask=1)
    choice = b.tune(reps=1)
    assert choice["sweep_width"] == 3
    b.run()
    z = b.results()
    for i, c in enumerate(circs):
        ref = z_of(O.run(c), c.n, 1)
        assert abs(z[i] - ref) <= 1e-12, (i, c.n, z[i], ref)
    b.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("fuse_w", [1, 2])
def test_batch_fusion_widths_match_oracle(dtype, fuse_w):
    """Each circuit's gates multiplied into blocks of at most 1 or 2 qubits
    (FP64 products, rounded once) before the batch program is built: final
    states and <Z_0> against the oracle, on ladder ansatz circuits (RY, RZ,
    CNOT ladder), random circuits with CNOTs and CZ layers, and a circuit
    with a doubly controlled gate (wider than the blocks, kept as is)."""
    circs = mixed_circuits(dtype, 24, seed=30 + fuse_w)
    wide = [C.Gate("H", (q,)) for q in range(6)] + [C.Gate("X", (5,), (0, 3)), C.Gate("RY", (2,), (), 0.7),
                                                   C.Gate("U1", (4,), (1, 2), 1.3), C.Gate("RZ", (2,), (), 0.2)]
    circs.append(C.Circuit(6, wide, 0, None, "toffoli"))
    b = sv.Batch(circs, dtype, z_mask=1, keep_states=True)
    b.config(13 if dtype == "c64" else 12, 4 if dtype == "c64" else 3, 64, fuse_w)
    b.run()
    z = b.results()
    for i, c in enumerate(circs):
        ref = O.run(c)
        got = b.state(i).astype(np.complex128)
        tol = C128_ATOL if dtype == "c128" else c64_bound(max(1, len(c)))
        assert np.max(np.abs(got - ref)) <= tol, (i, c.n, fuse_w)
        assert abs(z[i] - z_of(ref, c.n, 1)) <= 2 * tol, (i, c.n)
    b.close()


def test_batch_rejects_sweep_wider_than_narrowest_circuit():
    """A complex64 batch may not use 4-qubit sweeps with a 3-qubit circuit;
    the C entry point refuses such circuits (widths below 4 for complex64)."""
    with pytest.raises(sv.SVError):
        sv.Batch([C.random_circuit(3, 2, 0), C.random_circuit(8, 2, 1)], "c64")


def test_batched_workload_full_size_sampled():
    """4096 circuits, widths uniform in 10..20, 8 ladder-ansatz layers,
    complex64, one graph launch; <Z_0> of a sampled subset (including the
    widest circuits) against the oracle, every result in [-1, 1]."""
    circs = [c.bound() for c in C.config3(seed=0)]
    assert len(circs) == 4096
    b = sv.Batch(circs, "c64", z_mask=1)
    b.run()
    z = b.results()
    assert np.all(np.abs(z) <= 1.0 + 1e-5)
    rng = np.random.default_rng(0)
    widest = [i for i, c in enumerate(circs) if c.n == 20][:4]
    sample = sorted(set(widest) | set(int(i) for i in rng.choice(4096, size=28, replace=False)))
    for i in sample:
        c = circs[i]
        ref = z_of(O.run(c), c.n, 1)
        assert abs(z[i] - ref) <= 2 * c64_bound(len(c)), (i, c.n, z[i], ref)
    b.run()
    np.testing.assert_array_equal(b.results(), z)
    b.close()


def test_batch_rejects_bad_widths():
    with pytest.raises(sv.SVError):
        sv.Batch([C.random_circuit(2, 1, 0)], "c64")
    with pytest.raises(sv.SVError):
        sv.Batch([C.random_circuit(31, 1, 0)], "c64")
