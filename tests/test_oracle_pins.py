"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: printed
values of the paper (tests/golden), Kronecker-product unitaries (Sec. 1.3.2 /
Sec. 2.2 definition of a gate on a register), closed forms (H^n, QFT,
Bernstein-Vazirani), matrix exponentials, finite differences and the
parameter-shift identity.  None of these reuses the oracle's own loops.
"""

import math

import numpy as np
import pytest
import scipy.linalg

import circuits as C
import oracle as O
from conftest import read_golden

O.build(force=False)

PAULI = {
    "X": np.array([[0, 1], [1, 0]], complex),
    "Y": np.array([[0, -1j], [1j, 0]], complex),
    "Z": np.array([[1, 0], [0, -1]], complex),
}


def parse_matrix(row):
    name, r, c = row[0], int(row[1]), int(row[2])
    vals = [complex(float(a), float(b)) for a, b in (e.split(",") for e in row[3:])]
    return name, np.array(vals, complex).reshape(r, c)


# ---------------------------------------------------------------- gate table

def test_fixed_gates_match_paper_table():
    table = dict(parse_matrix(r) for r in read_golden("gate_table.txt"))
    for name in ("H", "X", "Y", "Z", "S", "T"):
        np.testing.assert_allclose(O.gate_matrix(name), table[name], atol=1e-15, rtol=0)


def test_cnot_matches_paper_table():
    """The table's CNOT (control = left factor, |c t>) equals the oracle's X on
    qubit 0 controlled by qubit 1, read column by column from basis states."""
    table = dict(parse_matrix(r) for r in read_golden("gate_table.txt"))
    full = np.zeros((4, 4), complex)
    for col in range(4):
        psi = O.basis_state(2, col)
        O.apply_1q(psi, 2, 0, O.gate_matrix("X"), ctrl=0b10)
        full[:, col] = psi
    np.testing.assert_array_equal(full, table["CNOT"])


@pytest.mark.parametrize("name", ["RX", "RY", "RZ"])
@pytest.mark.parametrize("theta", [0.0, 0.3, math.pi / 2, 2.5, math.pi, 5.9])
def test_rotations_are_exponentials(name, theta):
    P = PAULI[name[1]]
    expect = scipy.linalg.expm(-0.5j * theta * P)
    np.testing.assert_allclose(O.gate_matrix(name, theta), expect, atol=1e-14, rtol=0)
    # d/dtheta exp(-i theta P/2) = -(i/2) P exp(-i theta P/2)
    np.testing.assert_allclose(O.gate_dmatrix(name, theta), -0.5j * P @ expect, atol=1e-14, rtol=0)


@pytest.mark.parametrize("theta", [0.0, 0.7, math.pi / 4, math.pi / 2, math.pi, 4.0])
def test_u1_phase_gate(theta):
    expect = scipy.linalg.expm(1j * theta * np.diag([0.0, 1.0]))
    np.testing.assert_allclose(O.gate_matrix("U1", theta), expect, atol=1e-14, rtol=0)
    np.testing.assert_allclose(O.gate_dmatrix("U1", theta), 1j * np.diag([0.0, 1.0]) @ expect,
                               atol=1e-14, rtol=0)


def test_phase_family_identities():
    np.testing.assert_allclose(O.gate_matrix("U1", math.pi), O.gate_matrix("Z"), atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix("U1", math.pi / 2), O.gate_matrix("S"), atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix("U1", math.pi / 4), O.gate_matrix("T"), atol=1e-15)


# ------------------------------------------------------------ qubit ordering

def test_kron_example_ordering():
    rows = {r[0]: r[1:] for r in read_golden("kron_example.txt")}
    left, right = int(rows["left_factor_qubit"][0]), int(rows["right_factor_qubit"][0])
    # |1> (x) |0> = |2>
    psi = O.basis_state(2, 0)
    O.apply_1q(psi, 2, left, O.gate_matrix("X"))
    assert np.argmax(np.abs(psi)) == int(rows["basis_1_0_index"][0])
    # (alpha1, beta1) (x) (alpha2, beta2)
    rng = np.random.default_rng(5)
    u1, u2 = C.random_unitary(2, rng), C.random_unitary(2, rng)
    psi = O.basis_state(2, 0)
    O.apply_1q(psi, 2, left, u1)
    O.apply_1q(psi, 2, right, u2)
    a1, b1 = u1[:, 0]
    a2, b2 = u2[:, 0]
    np.testing.assert_allclose(psi, [a1 * a2, a1 * b2, b1 * a2, b1 * b2], atol=1e-15)


# ------------------------------------------------- full Kronecker unitaries

def kron_all(ops):
    """ops[q] is the 2x2 operator on qubit q; qubit n-1 is the left factor."""
    out = np.array([[1.0 + 0j]])
    for op in reversed(ops):
        out = np.kron(out, op)
    return out


def full_unitary(n, gate, mat):
    """2^n x 2^n matrix of a (controlled) k-qubit gate built from Kronecker
    products: sum over matrix entries U[r,c] of the tensor product of
    |r_j><c_j| on target j, identity elsewhere; controls via projectors."""
    eye = np.eye(2, dtype=complex)
    P1 = np.diag([0.0, 1.0]).astype(complex)
    k = len(gate.targets)
    dim = 1 << k
    G = np.zeros((1 << n, 1 << n), complex)
    for r in range(dim):
        for c in range(dim):
            if mat[r, c] == 0:
                continue
            ops = [eye] * n
            for j, q in enumerate(gate.targets):
                e = np.zeros((2, 2), complex)
                e[(r >> j) & 1, (c >> j) & 1] = 1.0
                ops[q] = e
            for q in gate.controls:
                ops[q] = P1
            G += mat[r, c] * kron_all(ops)
    if gate.controls:
        ops = [eye] * n
        for q in gate.controls:
            ops[q] = P1
        Pc = kron_all(ops)
        G += np.eye(1 << n) - Pc
    return G


def gate_mat(g):
    return g.matrix if g.name == "U" else O.gate_matrix(g.name, g.theta)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_random_circuit_matches_kronecker_product(n, seed):
    circ = C.random_circuit(n, 4, seed, "X", n // 2)
    U = np.eye(1 << n, dtype=complex)
    for g in circ.gates:
        U = full_unitary(n, g, gate_mat(g)) @ U
    psi = O.run(circ)
    np.testing.assert_allclose(psi, U[:, 0], atol=1e-12, rtol=0)


@pytest.mark.parametrize("k,controls", [(1, 2), (2, 0), (2, 1), (3, 1), (4, 0)])
def test_kqubit_unitaries_match_kronecker_product(k, controls):
    n = 7
    circ = C.random_unitary_gates(n, 6, k, seed=10 * k + controls, max_controls=controls)
    rng = np.random.default_rng(3)
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi0 /= np.linalg.norm(psi0)
    expect = psi0.copy()
    for g in circ.gates:
        expect = full_unitary(n, g, g.matrix) @ expect
    got = O.run_gates(n, circ.gates, psi0.copy())
    np.testing.assert_allclose(got, expect, atol=1e-12, rtol=0)


def test_multi_controlled_named_gates_match_kronecker_product():
    """Toffoli-like gates: a named one-qubit gate with two or three controls
    acts only where every control bit is 1."""
    n = 6
    rng = np.random.default_rng(21)
    gates = []
    for i in range(12):
        qs = [int(v) for v in rng.choice(n, size=4, replace=False)]
        name = ["X", "RY", "H", "U1"][i % 4]
        gates.append(C.Gate(name, (qs[0],), tuple(qs[1:2 + i % 3]), float(rng.uniform(0, 6.28))))
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi0 /= np.linalg.norm(psi0)
    expect = psi0.copy()
    for g in gates:
        expect = full_unitary(n, g, gate_mat(g)) @ expect
    got = O.run_gates(n, gates, psi0.copy())
    np.testing.assert_allclose(got, expect, atol=1e-12, rtol=0)


def test_config0_matches_kronecker_product():
    """Config-0 circuit at 8 qubits (same recipe, smaller register)."""
    circ = C.random_circuit(8, 20, 0, "X", 4)
    U = np.eye(1 << 8, dtype=complex)
    for g in circ.gates:
        U = full_unitary(8, g, gate_mat(g)) @ U
    np.testing.assert_allclose(O.run(circ), U[:, 0], atol=1e-12, rtol=0)


# ----------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 4, 9, 14])
def test_hadamard_all_from_zero_is_uniform(n):
    psi = O.basis_state(n, 0)
    for q in range(n):
        O.apply_1q(psi, n, q, O.gate_matrix("H"))
    np.testing.assert_allclose(psi, np.full(1 << n, 2.0 ** (-n / 2)), atol=1e-15, rtol=0)


@pytest.mark.parametrize("n,a", [(3, 5), (8, 0b10110001), (11, 1234)])
def test_hadamard_all_on_basis_state_signs(n, a):
    psi = O.basis_state(n, a)
    for q in range(n):
        O.apply_1q(psi, n, q, O.gate_matrix("H"))
    x = np.arange(1 << n)
    signs = np.array([(-1.0) ** bin(a & int(v)).count("1") for v in x])
    np.testing.assert_allclose(psi, signs * 2.0 ** (-n / 2), atol=1e-14, rtol=0)


def test_bernstein_vazirani_worked_example():
    rows = {r[0]: int(r[1]) for r in read_golden("bernstein_vazirani.txt")}
    n, a = rows["n_qubits"], rows["hidden"]
    psi = O.run(C.bernstein_vazirani(n, a))
    p, total = O.probabilities(psi, n)
    assert abs(total - 1.0) < 1e-12
    assert abs(p[a] - 1.0) < 1e-12
    assert np.sum(np.delete(p, a)) < 1e-20
    # every draw of the inverse-CDF sampler lands on the hidden integer
    u = np.random.default_rng(0).random(rows["samples"])
    draws = np.searchsorted(np.cumsum(p), u, side="right")
    assert np.all(draws == rows["outcome"])


def bit_reverse(x, n):
    return int(format(x, f"0{n}b")[::-1], 2)


def qft_closed_form(n, x, ys):
    """QFT circuit without swaps applied to |x>: amplitude of |y> is
    2^{-n/2} exp(2 pi i (rev_n(x) * y mod 2^n) / 2^n)."""
    r = bit_reverse(x, n)
    ph = (r * np.asarray(ys, dtype=object)) % (1 << n)
    ang = np.array([2.0 * math.pi * float(v) / float(1 << n) for v in ph])
    return np.exp(1j * ang) * 2.0 ** (-n / 2)


@pytest.mark.parametrize("n", [1, 2, 3, 6, 10])
def test_qft_of_basis_state_closed_form(n):
    rng = np.random.default_rng(n)
    xs = [0, (1 << n) - 1] + [int(v) for v in rng.integers(0, 1 << n, size=3)]
    for x in xs:
        psi = O.run(C.qft_circuit(n, x))
        np.testing.assert_allclose(psi, qft_closed_form(n, x, range(1 << n)), atol=1e-13, rtol=0)


# ------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", [0, 1])
def test_unit_norm_after_every_gate(seed):
    circ = C.config0(seed)
    psi = O.basis_state(circ.n, 0)
    for g in circ.gates:
        O.run_gates(circ.n, [g], psi)
        assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13


@pytest.mark.parametrize("maker", [lambda: C.config0(3), lambda: C.qft_circuit(9, 77),
                                   lambda: C.random_unitary_gates(9, 10, 2, 4, 2)])
def test_inverse_round_trip(maker):
    circ = maker()
    psi = O.run(circ)
    O.run(circ, psi=psi, inverse=True)
    np.testing.assert_allclose(psi, O.basis_state(circ.n, circ.basis), atol=1e-12, rtol=0)


def test_single_qubit_probabilities():
    rng = np.random.default_rng(1)
    u = C.random_unitary(2, rng)
    psi = O.basis_state(1, 0)
    O.apply_1q(psi, 1, 0, u)
    p, total = O.probabilities(psi, 1)
    alpha, beta = u[0, 0], u[1, 0]
    np.testing.assert_allclose(p, [abs(alpha) ** 2, abs(beta) ** 2], atol=1e-15)
    assert abs(total - 1.0) < 1e-15


# ------------------------------------------------------------ expectations

def z_string_matrix(n, mask):
    Z = np.diag([1.0, -1.0]).astype(complex)
    return kron_all([Z if (mask >> q) & 1 else np.eye(2) for q in range(n)])


def test_expectation_matches_kronecker_observable():
    n = 6
    circ = C.random_circuit(n, 5, 9, "X", 3)
    psi = O.run(circ)
    masks = [1, 0b101, 0b111111, 0b010010, 0]
    coeffs = [0.5, -1.25, 2.0, 0.75, 0.1]
    H = sum(c * z_string_matrix(n, m) for m, c in zip(masks, coeffs))
    expect = np.vdot(psi, H @ psi).real
    assert abs(O.expectation_z(psi, n, masks, coeffs) - expect) < 1e-13


@pytest.mark.parametrize("x", [0, 5, 0b101101])
def test_expectation_on_basis_states(x):
    n = 6
    psi = O.basis_state(n, x)
    for q in range(n):
        assert O.expectation_z(psi, n, [1 << q], [1.0]) == 1.0 - 2.0 * ((x >> q) & 1)


@pytest.mark.parametrize("theta", [0.0, 0.4, 1.9, math.pi, 5.1])
def test_ry_expectation_cosine(theta):
    psi = O.basis_state(1, 0)
    O.apply_1q(psi, 1, 0, O.gate_matrix("RY", theta))
    assert abs(O.expectation_z(psi, 1, [1], [1.0]) - math.cos(theta)) < 1e-15


def test_hea_layer_without_entanglers():
    """One RY/RZ layer: <Z_q> = cos(theta_RY on q); RZ does not change it."""
    n = 5
    circ = C.hea_circuit(n, 1, 4, "ladder")
    gates = [g for g in circ.bound().gates if not g.controls]
    psi = O.run_gates(n, gates, O.basis_state(n, 0))
    for q in range(n):
        assert abs(O.expectation_z(psi, n, [1 << q], [1.0]) - math.cos(circ.params[2 * q])) < 1e-14


# ----------------------------------------------------------------- adjoint

def shifted(params, i, d):
    p = params.copy()
    p[i] += d
    return p


@pytest.mark.parametrize("entangler,n,layers", [("ring", 4, 2), ("ladder", 5, 2), ("ring", 6, 1)])
def test_adjoint_against_parameter_shift_and_fd(entangler, n, layers):
    circ = C.hea_circuit(n, layers, 7, entangler)
    masks, coeffs = C.zz_ring_observable(n)
    L, grad = O.adjoint_grad(circ, circ.params, masks, coeffs)
    assert abs(L - O.loss(circ, circ.params, masks, coeffs)) < 1e-13
    h = 1e-6
    for i in range(len(circ.params)):
        ps = 0.5 * (O.loss(circ, shifted(circ.params, i, math.pi / 2), masks, coeffs)
                    - O.loss(circ, shifted(circ.params, i, -math.pi / 2), masks, coeffs))
        fd = (O.loss(circ, shifted(circ.params, i, h), masks, coeffs)
              - O.loss(circ, shifted(circ.params, i, -h), masks, coeffs)) / (2 * h)
        assert abs(grad[i] - ps) < 1e-12, (i, grad[i], ps)
        assert abs(grad[i] - fd) < 1e-7, (i, grad[i], fd)


def test_adjoint_controlled_phase_and_rx_against_fd():
    """Parametrised controlled-U1 and RX gates (derivative zero outside the
    control subspace), observable with mixed coefficients."""
    n = 5
    rng = np.random.default_rng(11)
    params = rng.uniform(0, 2 * math.pi, 6)
    gates = [C.Gate("H", (q,)) for q in range(n)]
    gates += [C.Gate("RX", (0,), (), 0.0, 0), C.Gate("U1", (1,), (3,), 0.0, 1),
              C.Gate("X", (2,), (0,)), C.Gate("RY", (4,), (1,), 0.0, 2),
              C.Gate("U1", (2,), (), 0.0, 3), C.Gate("RZ", (3,), (4,), 0.0, 4),
              C.Gate("RX", (1,), (), 0.0, 5), C.Gate("RX", (0,), (), 0.0, 5)]
    circ = C.Circuit(n, gates, 0, params)
    masks, coeffs = [0b00011, 0b10100, 0b01000, 0b11111], [1.0, -0.5, 0.25, 2.0]
    L, grad = O.adjoint_grad(circ, params, masks, coeffs)
    h = 1e-6
    for i in range(len(params)):
        fd = (O.loss(circ, shifted(params, i, h), masks, coeffs)
              - O.loss(circ, shifted(params, i, -h), masks, coeffs)) / (2 * h)
        assert abs(grad[i] - fd) < 1e-7, (i, grad[i], fd)
