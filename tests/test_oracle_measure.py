"""Pins of the oracle's measurement functions (marginals, collapse,
outcome selection, sampling) against what the paper and the mathematics fix:
the single-qubit example and the post-measurement state of Sec. 1.3.3, the
Bernstein-Vazirani outcome of App. C, closed forms for product and Bell
states, the chain rule of sequential measurement, marginals computed by an
independent tensor reduction, and the inverse-CDF rule on hand-built
distributions."""

import numpy as np
import pytest

import circuits as C
import oracle as O
from conftest import read_golden


def _random_state(n, seed):
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return np.ascontiguousarray(psi / np.linalg.norm(psi))


def _tensor_marginals(psi, n, mask):
    """|psi|^2 as an n-axis tensor (axis i <-> qubit n-1-i), summed over the
    qubits outside mask; outcome bit i = i-th lowest qubit of mask."""
    p = (np.abs(psi) ** 2).reshape([2] * n)
    qs = [q for q in range(n) if (mask >> q) & 1]
    other = tuple(n - 1 - q for q in range(n) if not (mask >> q) & 1)
    m = p.sum(axis=other) if other else p
    # remaining axes are the mask qubits in descending order; flatten so that
    # the lowest mask qubit is the least significant outcome bit
    return m.reshape(-1) if len(qs) else np.array([m.sum()])


def test_select_hand_distribution():
    p = np.array([0.1, 0.2, 0.3, 0.4])
    # cumulative 0.1, 0.3, 0.6, 1.0: smallest i with c_i > u
    for u, want in [(0.0, 0), (0.05, 0), (0.15, 1), (0.29, 1), (0.35, 2), (0.59, 2), (0.65, 3), (0.999, 3)]:
        assert O.select(p, u) == want, u
    # zero-probability outcomes are never selected
    z = np.array([0.0, 0.5, 0.0, 0.5])
    assert [O.select(z, u) for u in (0.0, 0.25, 0.5, 0.75)] == [1, 1, 3, 3]
    # unnormalised weights select by their share of the total
    w = np.array([2.0, 6.0])
    assert O.select(w, 0.2) == 0 and O.select(w, 0.3) == 1


def test_select_matches_searchsorted():
    rng = np.random.default_rng(3)
    for m in (1, 2, 7, 64):
        p = rng.random(m)
        p[rng.random(m) < 0.3] = 0.0
        if p.sum() == 0:
            p[0] = 1.0
        c = np.cumsum(p)
        for u in rng.random(200):
            want = int(np.searchsorted(c, u * c[-1], side="right"))
            assert O.select(p, u) == want


@pytest.mark.parametrize("mask", [0b1, 0b100000, 0b10110, 0b111111, 0b101001])
def test_marginals_match_tensor_reduction(mask):
    n = 6
    psi = _random_state(n, 11)
    got = O.marginals(psi, n, mask)
    want = _tensor_marginals(psi, n, mask)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)
    assert abs(got.sum() - 1.0) < 1e-13


def test_marginals_product_state_closed_form():
    # |psi> = U_{n-1} (x) ... (x) U_0 |0...0>: qubit q is U_q|0> = (U_q[0,0], U_q[1,0])
    n = 5
    us = [C.random_unitary(2, np.random.default_rng(100 + q)) for q in range(n)]
    gates = [C.Gate("U", (q,), matrix=us[q]) for q in range(n)]
    psi = O.run_gates(n, gates, O.basis_state(n, 0))
    for q in range(n):
        pq = O.marginals(psi, n, 1 << q)
        np.testing.assert_allclose(pq, [abs(us[q][0, 0]) ** 2, abs(us[q][1, 0]) ** 2], atol=1e-14)
    # two qubits: the product of the single-qubit marginals, outcome bit 0 = lower qubit
    p13 = O.marginals(psi, n, (1 << 1) | (1 << 3))
    a = [abs(us[1][0, 0]) ** 2, abs(us[1][1, 0]) ** 2]
    b = [abs(us[3][0, 0]) ** 2, abs(us[3][1, 0]) ** 2]
    np.testing.assert_allclose(p13, [a[0] * b[0], a[1] * b[0], a[0] * b[1], a[1] * b[1]], atol=1e-14)


def test_collapse_single_qubit_example():
    # Sec. 1.3.3: alpha|0> + beta|1>; p(0) = |alpha|^2 and the state becomes
    # (alpha/|alpha|)|0>, p(1) = |beta|^2 and (beta/|beta|)|1>
    alpha, beta = 0.6 * np.exp(0.4j), 0.8 * np.exp(-1.1j)
    for value, amp, p in [(0, alpha, 0.36), (1, beta, 0.64)]:
        psi = np.array([alpha, beta], np.complex128)
        got = O.collapse(psi, 1, 1, value)
        assert abs(got - p) < 1e-15
        want = np.zeros(2, np.complex128)
        want[value] = amp / abs(amp)
        np.testing.assert_allclose(psi, want, atol=1e-15)


def test_collapse_zero_probability_leaves_state():
    psi = O.basis_state(3, 5)
    keep = psi.copy()
    assert O.collapse(psi, 3, 0b010, 0b010) == 0.0
    np.testing.assert_array_equal(psi, keep)


def test_measure_bell_state():
    # H(0), CNOT(0 -> 1): (|00> + |11>)/sqrt(2); measuring qubit 0 fixes qubit 1
    gates = [C.Gate("H", (0,)), C.Gate("X", (1,), controls=(0,))]
    for u, bit in [(0.2, 0), (0.7, 1)]:
        psi = O.run_gates(2, gates, O.basis_state(2, 0))
        value, p = O.measure(psi, 2, 0b01, u)
        assert value == bit and abs(p - 0.5) < 1e-15
        want = np.zeros(4, np.complex128)
        want[3 * bit] = 1.0
        np.testing.assert_allclose(psi, want, atol=1e-15)
        assert np.allclose(O.marginals(psi, 2, 0b10), [1 - bit, bit])


def test_sequential_measurement_chain_rule():
    # P(A = a, B = b) = P(A = a) P(B = b | A = a): measuring A then B on the
    # collapsed state reproduces the joint marginal of A u B
    n, ma, mb = 6, 0b001001, 0b100100
    psi = _random_state(n, 5)
    joint = O.marginals(psi, n, ma | mb)  # outcome bits: qubits 0, 2, 3, 5
    pa = O.marginals(psi, n, ma)          # bits: qubits 0, 3
    for a in range(4):
        phi = psi.copy()
        va = (a & 1) | ((a >> 1) << 3)
        pr = O.collapse(phi, n, ma, va)
        assert abs(pr - pa[a]) < 1e-14
        pb = O.marginals(phi, n, mb)      # bits: qubits 2, 5
        for b in range(4):
            q0, q3 = a & 1, a >> 1
            q2, q5 = b & 1, b >> 1
            j = q0 | (q2 << 1) | (q3 << 2) | (q5 << 3)
            assert abs(pa[a] * pb[b] - joint[j]) < 1e-14


def test_measure_basis_state_is_certain():
    n, x = 7, 0b1011001
    psi = O.basis_state(n, x)
    value, p = O.measure(psi, n, (1 << n) - 1, 0.77)
    assert value == x and p == 1.0
    np.testing.assert_array_equal(psi, O.basis_state(n, x))


def test_sample_bernstein_vazirani():
    rows = {r[0]: int(r[1]) for r in read_golden("bernstein_vazirani.txt")}
    n, a, s = rows["n_qubits"], rows["hidden"], rows["samples"]
    psi = O.run(C.bernstein_vazirani(n, a))
    out = O.sample(psi, n, C.uniforms(s, 7))
    assert np.all(out == rows["outcome"])


def test_sample_chi_square():
    n, s = 4, 40000
    psi = _random_state(n, 9)
    p = np.abs(psi) ** 2
    out = O.sample(psi, n, C.uniforms(s, 21))
    counts = np.bincount(out.astype(np.int64), minlength=1 << n)
    chi2 = float(((counts - s * p) ** 2 / (s * p)).sum())
    assert chi2 < 42.6  # 15 degrees of freedom, upper 1e-4 tail


def test_sample_does_not_change_state():
    psi = _random_state(5, 2)
    keep = psi.copy()
    O.sample(psi, 5, C.uniforms(10, 1))
    np.testing.assert_array_equal(psi, keep)
