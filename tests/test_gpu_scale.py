"""Parity at the benchmark's full sizes (30 qubits complex128, 32 qubits
complex64, and the 30-qubit fusion workload) in the launch configuration the
benchmark times, on outputs computable independently of the full state:

* the QFT of a random basis state against its closed form on sampled
  amplitudes (the headline workload's first circuit);
* block-product circuits (random layers whose entanglers stay inside fixed
  qubit blocks): every amplitude is a product of small block amplitudes the
  oracle computes, so sampled amplitudes of the full state are checked one by
  one, for the tile-pass path and for the fused path.
Tolerances: complex128 within 1e-12 per amplitude; complex64 within the
rigorous 2-norm bound 4 sqrt(2) eps32 G (helpers.c64_bound) per amplitude,
and a sampled relative 2-norm error sqrt(sum |d|^2 / sum |ref|^2) below 1e-5
(the per-gate FP32 rounding, 6e-8, grows like sqrt(G) for G ~ 10^3 gates;
single amplitudes near zero may carry larger relative errors)."""

import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from helpers import C128_ATOL, c64_bound

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1805_00988_amd as sv  # noqa: E402

O.build(force=False)

SIZES = [("c128", 30), ("c64", 32)]


def sample_indices(n, count, seed):
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, 1 << n, size=count, dtype=np.int64))


def gpu_amplitudes(st, idx):
    return st.amps[torch.from_numpy(idx).to(st.amps.device)].cpu().numpy().astype(np.complex128)


def check(got, ref, dtype, n_gates):
    err = np.abs(got - ref)
    if dtype == "c128":
        assert err.max() <= C128_ATOL, err.max()
    else:
        assert err.max() <= c64_bound(n_gates), err.max()
        assert rel_norm(err, ref) < 1e-5


def rel_norm(err, ref):
    return math.sqrt(float(np.sum(err ** 2)) / float(np.sum(np.abs(ref) ** 2)))


def bit_reverse(x, n):
    return int(format(x, f"0{n}b")[::-1], 2)


@pytest.mark.parametrize("dtype,n", SIZES)
def test_qft_full_size_closed_form(dtype, n):
    x = C.random_basis(n, 5)
    circ = C.qft_circuit(n, x)
    st = sv.State(n, dtype).set_basis(x)
    st.run(circ.gates, mode=sv.SV_RUN_TILED)
    idx = sample_indices(n, 4096, 17)
    r = bit_reverse(x, n)
    ph = np.array([(r * int(y)) % (1 << n) for y in idx], dtype=np.float64)
    ref = np.exp(2j * math.pi * ph / float(1 << n)) * 2.0 ** (-n / 2)
    check(gpu_amplitudes(st, idx), ref, dtype, len(circ))
    assert abs(st.probabilities() - 1.0) < (1e-12 if dtype == "c128" else 1e-5)
    del st
    torch.cuda.empty_cache()


def block_reference(circ, blocks, idx):
    """Amplitudes at idx of a block-product circuit from per-block oracle runs."""
    amps = np.ones(len(idx), np.complex128)
    for qs in blocks:
        local = {q: j for j, q in enumerate(qs)}
        sub = [C.Gate(g.name, tuple(local[q] for q in g.targets), tuple(local[q] for q in g.controls),
                      g.theta, g.param, g.matrix)
               for g in circ.gates if all(q in local for q in g.qubits)]
        psi = O.run_gates(len(qs), sub, O.basis_state(len(qs), 0))
        li = np.zeros(len(idx), np.int64)
        for j, q in enumerate(qs):
            li |= ((idx >> q) & 1) << j
        amps *= psi[li]
    return amps


@pytest.mark.parametrize("dtype,n", SIZES)
def test_block_product_full_size_tiled(dtype, n):
    circ, blocks = C.block_product_circuit(n, 6, 20, seed=3)
    st = sv.State(n, dtype).run(circ.gates, mode=sv.SV_RUN_TILED)
    idx = sample_indices(n, 4096, 23)
    check(gpu_amplitudes(st, idx), block_reference(circ, blocks, idx), dtype, len(circ))
    del st
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,k", [(sv.SV_PREC_SPLIT_BF16, 4), (sv.SV_PREC_FP32, 4), (sv.SV_PREC_SPLIT_BF16, 5)])
def test_block_product_full_size_fused(prec, k):
    """The fusion workload's size (30 qubits, complex64) through fused tile
    passes; per-amplitude bound of the fused arithmetic: the FP32 2-norm bound
    for the block count plus 2^k 2^-15 per block for split-BF16 operands."""
    n = 30
    circ, blocks = C.block_product_circuit(n, 6, 40, seed=4)
    st = sv.State(n, "c64")
    nb = st.run_fused(circ.gates, k_max=k, prec=prec)
    idx = sample_indices(n, 4096, 29)
    got = gpu_amplitudes(st, idx)
    ref = block_reference(circ, blocks, idx)
    per = (2 ** k) * (2.0 ** -15 if prec == sv.SV_PREC_SPLIT_BF16 else 4 * 2.0 ** -24)
    err = np.abs(got - ref)
    assert err.max() <= nb * per, (err.max(), nb)
    assert rel_norm(err, ref) < 1e-4
    del st
    torch.cuda.empty_cache()
