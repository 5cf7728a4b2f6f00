"""GPU parity of the plain gate path against the FP64 oracle.

Every case runs the HIP kernels through the C-ABI (via the Python binding)
and the oracle on the same seeded input, and compares element by element.
Sizes span one vector, several LDS tiles (tiles hold 2^12 / 2^13
amplitudes) and ragged launch tails (pair counts below one workgroup's
share)."""

import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from helpers import assert_state_close, random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1805_00988_amd as sv  # noqa: E402

O.build(force=False)

DTYPES = ["c128", "c64"]
NP_DT = {"c128": np.complex128, "c64": np.complex64}


def gpu_state(n, dtype, psi0=None):
    st = sv.State(n, dtype)
    if psi0 is not None:
        st.amps.copy_(torch.from_numpy(psi0.astype(NP_DT[dtype])))
    return st


def oracle_input(psi0, dtype):
    """The exact values the GPU starts from, widened to complex128."""
    return psi0.astype(NP_DT[dtype]).astype(np.complex128)


def run_both(n, dtype, gates, seed, mode):
    psi0 = random_state(n, seed)
    st = gpu_state(n, dtype, psi0)
    st.run(gates, mode=mode)
    got = st.numpy()
    ref = O.run_gates(n, gates, oracle_input(psi0, dtype))
    return got, ref


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 3, 7, 14])
def test_one_qubit_gate_every_target(dtype, n):
    rng = np.random.default_rng(100 + n)
    for t in range(n):
        U = C.random_unitary(2, rng)
        g = C.Gate("U", (t,), (), 0.0, -1, U)
        got, ref = run_both(n, dtype, [g], seed=t, mode=sv.SV_RUN_PER_GATE)
        assert_state_close(got, ref, dtype, 1)


@pytest.mark.parametrize("dtype", DTYPES)
def test_controlled_gates(dtype):
    n = 13
    rng = np.random.default_rng(7)
    cases = []
    for t in range(n):
        for nc in (1, 2, 3):
            others = [q for q in range(n) if q != t]
            ctrl = tuple(int(c) for c in rng.choice(others, size=nc, replace=False))
            cases.append((t, ctrl))
    cases += [(5, (0,)), (0, (1,)), (1, (0,)), (12, (0, 1)), (3, (0, 12, 7, 9, 11))]
    for i, (t, ctrl) in enumerate(cases):
        g = C.Gate("U", (t,), ctrl, 0.0, -1, C.random_unitary(2, rng))
        got, ref = run_both(n, dtype, [g], seed=i, mode=sv.SV_RUN_PER_GATE)
        assert_state_close(got, ref, dtype, 1)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [9, 16])
def test_multi_controlled_gates_tiled(dtype, n):
    """Tile passes of gates with 0-3 controls of every kind (general, real,
    real-diagonal/imaginary-off-diagonal, exchange, diagonal, 4x4), so that
    controls fall on register positions, on lane bits and on qubits outside
    the tile, against the oracle."""
    rng = np.random.default_rng(40 + n)
    gates = []
    for i in range(180):
        nc = int(rng.integers(0, 4))
        two = i % 9 == 8
        qs = [int(q) for q in rng.choice(n, size=(2 if two else 1) + nc, replace=False)]
        ctrl = tuple(qs[2 if two else 1:])
        if two:
            gates.append(C.Gate("U", (qs[0], qs[1]), ctrl, 0.0, -1, C.random_unitary(4, rng)))
            continue
        name = ["U", "H", "RX", "X", "Y", "T", "RZ", "RY"][int(rng.integers(0, 8))]
        th = float(rng.uniform(0, 6.28))
        if name == "U":
            gates.append(C.Gate("U", (qs[0],), ctrl, 0.0, -1, C.random_unitary(2, rng)))
        else:
            gates.append(C.Gate(name, (qs[0],), ctrl, th if name in ("RX", "RZ", "RY") else None))
    got, ref = run_both(n, dtype, gates, seed=41, mode=sv.SV_RUN_TILED)
    assert_state_close(got, ref, dtype, len(gates))


@pytest.mark.parametrize("dtype", DTYPES)
def test_many_controls_streamed(dtype):
    """Gates with 10 to 13 controls at 16 qubits, one launch per gate: the
    streamed kernels enumerate at most 10 inserted bit positions (target and
    controls) and test the remaining control bits per element.  General,
    phase (subspace) and two-qubit gates, controls above and below their
    targets, against the oracle."""
    n = 16
    rng = np.random.default_rng(77)
    gates = [C.Gate("H", (q,)) for q in range(n)]
    for i in range(12):
        nc = 10 + i % 4
        two = i % 3 == 2
        qs = [int(q) for q in rng.choice(n, size=nc + (2 if two else 1), replace=False)]
        tg = tuple(qs[:2] if two else qs[:1])
        ctrl = tuple(qs[len(tg):])
        if two:
            gates.append(C.Gate("U", tg, ctrl, 0.0, -1, C.random_unitary(4, rng)))
        elif i % 3 == 1:
            gates.append(C.Gate("U1", tg, ctrl, float(rng.uniform(0, 6.28))))
        else:
            gates.append(C.Gate("U", tg, ctrl, 0.0, -1, C.random_unitary(2, rng)))
    got, ref = run_both(n, dtype, gates, seed=78, mode=sv.SV_RUN_PER_GATE)
    assert_state_close(got, ref, dtype, len(gates))
    # the controls must have acted: the controlled part changes the state
    plain = O.run_gates(n, gates[:n], oracle_input(random_state(n, 78), dtype))
    assert np.max(np.abs(ref - plain)) > 1e-6


@pytest.mark.parametrize("dtype", DTYPES)
def test_two_qubit_gates_all_pairs(dtype):
    n = 6
    rng = np.random.default_rng(8)
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            g = C.Gate("U", (a, b), (), 0.0, -1, C.random_unitary(4, rng))
            got, ref = run_both(n, dtype, [g], seed=a * n + b, mode=sv.SV_RUN_PER_GATE)
            assert_state_close(got, ref, dtype, 1)


@pytest.mark.parametrize("dtype", DTYPES)
def test_two_qubit_gates_controlled_large(dtype):
    n = 15
    circ = C.random_unitary_gates(n, 24, 2, seed=9, max_controls=2)
    circ.gates += [C.Gate("U", (0, 14), (3,), 0.0, -1, C.random_unitary(4, np.random.default_rng(1))),
                   C.Gate("U", (13, 0), (), 0.0, -1, C.random_unitary(4, np.random.default_rng(2)))]
    for mode in (sv.SV_RUN_PER_GATE, sv.SV_RUN_TILED):
        got, ref = run_both(n, dtype, circ.gates, seed=3, mode=mode)
        assert_state_close(got, ref, dtype, len(circ.gates))


@pytest.mark.parametrize("dtype", DTYPES)
def test_diagonal_and_phase_gates(dtype):
    n = 12
    gates = []
    rng = np.random.default_rng(4)
    for t in range(n):
        gates.append(C.Gate("U1", (t,), ((t + 3) % n,), float(rng.uniform(0, 6.28))))
        gates.append(C.Gate(["Z", "S", "T"][t % 3], (t,)))
        gates.append(C.Gate("RZ", (t,), (), float(rng.uniform(0, 6.28))))
        gates.append(C.Gate("U1", (t,), (), float(rng.uniform(0, 6.28))))
    gates.append(C.Gate("U1", (0,), (1, 2), 1.1))
    gates.append(C.Gate("Z", (1,), (0,)))
    for mode in (sv.SV_RUN_PER_GATE, sv.SV_RUN_TILED):
        got, ref = run_both(n, dtype, gates, seed=5, mode=mode)
        assert_state_close(got, ref, dtype, len(gates))


def phase_run_circuit(n, n_phase, seed):
    """Hadamards on every qubit, then runs of phase gates (U1, Z, S, T with
    0-2 controls on random qubits, so that their conditions fall on register
    positions, lane bits and qubits outside the tile), broken by an RZ or an
    RX now and then (runs of 1 to 12 gates), then Hadamards again."""
    rng = np.random.default_rng(seed)
    gates = [C.Gate("H", (q,)) for q in range(n)]
    left = n_phase
    while left > 0:
        run = int(min(left, rng.integers(1, 13)))
        for _ in range(run):
            qs = rng.choice(n, size=1 + int(rng.integers(0, 3)), replace=False)
            name = ["U1", "Z", "S", "T"][int(rng.integers(0, 4))]
            theta = float(rng.uniform(0, 6.28)) if name == "U1" else None
            gates.append(C.Gate(name, (int(qs[0]),), tuple(int(q) for q in qs[1:]), theta))
        left -= run
        t = int(rng.integers(0, n))
        gates.append(C.Gate(["RZ", "RX"][int(rng.integers(0, 2))], (t,), (), float(rng.uniform(0, 6.28))))
    gates += [C.Gate("H", (q,)) for q in range(n)]
    return gates


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [5, 14, 17])
def test_phase_runs_tiled(dtype, n):
    """Runs of commuting phase gates, gathered into per-lane factors by the
    tile pass, against the oracle's gate-by-gate application."""
    gates = phase_run_circuit(n, 160, seed=20 + n)
    got, ref = run_both(n, dtype, gates, seed=21, mode=sv.SV_RUN_TILED)
    assert_state_close(got, ref, dtype, len(gates))


def outside_diagonal_circuit(n, seed, layers=8):
    """Dense gates on the low qubits only (so that tile passes hold the low
    qubits) mixed with diagonal gates anywhere: uncontrolled RZ, Z, S, T,
    phase gates with 0-3 controls, and controlled RZ, in runs of 1 to 8."""
    rng = np.random.default_rng(seed)
    lowq = max(1, n // 2)
    gates = [C.Gate("H", (q,)) for q in range(n)]
    for _ in range(layers):
        for q in range(lowq):
            gates.append(C.Gate(["H", "RX", "RY"][int(rng.integers(0, 3))], (q,), (), float(rng.uniform(0, 6.28))))
        for _ in range(int(rng.integers(1, 9))):
            qs = [int(x) for x in rng.choice(n, size=1 + int(rng.integers(0, 4)), replace=False)]
            kind = int(rng.integers(0, 4))
            th = float(rng.uniform(0, 6.28))
            if kind == 0:
                gates.append(C.Gate(["RZ", "Z", "S", "T"][int(rng.integers(0, 4))], (qs[0],), (), th))
            elif kind == 1:
                gates.append(C.Gate("U1", (qs[0],), tuple(qs[1:]), th))
            elif kind == 2:
                gates.append(C.Gate(["Z", "S", "T"][int(rng.integers(0, 3))], (qs[0],), tuple(qs[1:])))
            else:
                gates.append(C.Gate("RZ", (qs[0],), tuple(qs[1:2]), th))
    gates += [C.Gate("H", (q,)) for q in range(n)]
    return gates


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [8, 16, 18])
def test_diagonal_gates_outside_tile(dtype, n):
    """Tile passes take phase gates and uncontrolled diagonal gates whatever
    the tile holds (the target outside the tile gives a factor per tile, a
    phase gate's target may move to one of its controls)."""
    gates = outside_diagonal_circuit(n, 90 + n)
    got, ref = run_both(n, dtype, gates, seed=11, mode=sv.SV_RUN_TILED)
    assert_state_close(got, ref, dtype, len(gates))


def phase_table_circuit(n, seed, layers=6):
    """Dense gates on qubits 0-5 between long runs of phase gates whose
    targets sit on low qubits and whose controls lie on high qubits: pairs of
    nearby high controls (gathered into tables over windows of index bits),
    controls far apart (left as single conditions), no control (constant
    factors), and phase gates on high targets alone."""
    rng = np.random.default_rng(seed)
    hi = list(range(n // 2, n))
    gates = [C.Gate("H", (q,)) for q in range(n)]
    for _ in range(layers):
        for q in range(6):
            gates.append(C.Gate(["H", "RX", "RY"][int(rng.integers(0, 3))], (q,), (), float(rng.uniform(0, 6.28))))
        for _ in range(40):
            t = int(rng.integers(0, 2))
            kind = int(rng.integers(0, 5))
            th = float(rng.uniform(0, 6.28))
            if kind == 0:
                c = int(rng.choice(hi))
                gates.append(C.Gate("U1", (t,), (c,), th))
            elif kind == 1:
                c0 = int(rng.choice(hi[:-3]))
                c1 = c0 + 1 + int(rng.integers(0, 3))
                gates.append(C.Gate("U1", (t,), (c0, c1), th))
            elif kind == 2:
                gates.append(C.Gate("U1", (t,), (hi[0], hi[-1]), th))
            elif kind == 3:
                gates.append(C.Gate(["S", "T", "Z"][int(rng.integers(0, 3))], (t,)))
            else:
                gates.append(C.Gate("U1", (int(rng.choice(hi)),), (), th))
    gates += [C.Gate("H", (q,)) for q in range(n)]
    return gates


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [14, 19, 22])
def test_phase_tables_outside_tile(dtype, n):
    """Gathered phases conditioned on qubits outside the tile: the factor per
    tile comes from tables over windows of index bits (products formed once
    on the host) and from single conditions; against the oracle's gate by
    gate application."""
    gates = phase_table_circuit(n, 300 + n)
    got, ref = run_both(n, dtype, gates, seed=12, mode=sv.SV_RUN_TILED)
    assert_state_close(got, ref, dtype, len(gates))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("mode", ["per_gate", "tiled"])
def test_config0_random_circuit(dtype, mode):
    """Config 0 recipe (12 qubits from |0>, depth 20, 6 CNOTs per layer)."""
    circ = C.config0(0)
    st = sv.State(circ.n, dtype)
    st.run(circ.gates, mode=sv.SV_RUN_TILED if mode == "tiled" else sv.SV_RUN_PER_GATE)
    assert_state_close(st.numpy(), O.run(circ), dtype, len(circ))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [3, 9, 13, 16, 18])
def test_random_circuits_tiled_vs_oracle(dtype, n):
    circ = C.random_circuit(n, 12, seed=n, entangler="X")
    st = sv.State(n, dtype)
    st.run(circ.gates, mode=sv.SV_RUN_TILED)
    assert_state_close(st.numpy(), O.run(circ), dtype, len(circ))


@pytest.mark.parametrize("dtype", DTYPES)
def test_cz_layers_tiled(dtype):
    circ = C.config2(n=17, seed=1, depth=8)
    st = sv.State(circ.n, dtype)
    st.run(circ.gates, mode=sv.SV_RUN_TILED)
    assert_state_close(st.numpy(), O.run(circ), dtype, len(circ))


def bit_reverse(x, n):
    return int(format(x, f"0{n}b")[::-1], 2)


def qft_reference(n, x, ys):
    r = bit_reverse(x, n)
    ph = [(r * int(y)) % (1 << n) for y in ys]
    return np.exp(1j * 2.0 * math.pi * np.array(ph, dtype=np.float64) / float(1 << n)) * 2.0 ** (-n / 2)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("mode", ["per_gate", "tiled"])
def test_qft_basis_state_closed_form(dtype, mode):
    n = 15
    x = C.random_basis(n, 11)
    circ = C.qft_circuit(n, x)
    st = sv.State(n, dtype).set_basis(x)
    st.run(circ.gates, mode=sv.SV_RUN_TILED if mode == "tiled" else sv.SV_RUN_PER_GATE)
    got = st.numpy()
    ref = qft_reference(n, x, range(1 << n))
    assert_state_close(got, ref, dtype, len(circ))
    assert_state_close(got, O.run(circ), dtype, len(circ))


@pytest.mark.parametrize("dtype", DTYPES)
def test_bernstein_vazirani(dtype):
    n, a = 14, 101
    st = sv.State(n, dtype).run(C.bernstein_vazirani(n, a).gates)
    p = torch.empty(1 << n, dtype=torch.float32 if dtype == "c64" else torch.float64, device="cuda")
    total = st.probabilities(p)
    p = p.cpu().numpy()
    assert abs(p[a] - 1.0) < 1e-6 and abs(total - 1.0) < 1e-6
    assert int(np.argmax(p)) == a


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 5, 12, 17])
def test_probabilities_match_oracle(dtype, n):
    circ = C.random_circuit(n, 6, seed=20 + n, entangler="X")
    st = sv.State(n, dtype).run(circ.gates)
    p = torch.empty(1 << n, dtype=torch.float32 if dtype == "c64" else torch.float64, device="cuda")
    total = st.probabilities(p)
    amps = st.numpy().astype(np.complex128)
    # reference from the GPU's own amplitudes (isolates the reduction) and
    # from the oracle state (end to end)
    p_ref, t_ref = O.probabilities(amps, n)
    got = p.cpu().numpy().astype(np.float64)
    if dtype == "c128":
        np.testing.assert_allclose(got, p_ref, rtol=0, atol=1e-15)
        assert abs(total - t_ref) < 1e-13
    else:
        np.testing.assert_allclose(got, p_ref, rtol=4 * 2.0 ** -24, atol=1e-30)
        assert abs(total - t_ref) < 1e-12
    p_orc, _ = O.probabilities(O.run(circ), n)
    np.testing.assert_allclose(got, p_orc, rtol=0, atol=1e-12 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [2, 10, 16])
def test_expectation_match_oracle(dtype, n):
    circ = C.random_circuit(n, 5, seed=40 + n, entangler="X")
    st = sv.State(n, dtype).run(circ.gates)
    rng = np.random.default_rng(n)
    masks = [int(m) for m in rng.integers(0, 1 << n, size=9)] + [1, (1 << n) - 1, 0]
    coeffs = [float(c) for c in rng.standard_normal(len(masks))]
    got = st.expectation(masks, coeffs)
    amps = st.numpy().astype(np.complex128)
    ref_same_input = O.expectation_z(amps, n, masks, coeffs)
    tol = 1e-12 if dtype == "c128" else 1e-10
    assert abs(got - ref_same_input) <= tol * max(1.0, sum(abs(c) for c in coeffs))
    ref = O.expectation_z(O.run(circ), n, masks, coeffs)
    assert abs(got - ref) <= (1e-11 if dtype == "c128" else 1e-4) * sum(abs(c) for c in coeffs)


@pytest.mark.parametrize("dtype", DTYPES)
def test_invalid_arguments_leave_state_unchanged(dtype):
    n = 8
    psi0 = random_state(n, 1)
    st = gpu_state(n, dtype, psi0)
    before = st.numpy().copy()
    with pytest.raises(sv.SVError):
        st.apply(np.eye(2), [n])            # target out of range
    with pytest.raises(sv.SVError):
        st.apply(np.eye(2), [3], [3])       # control equals target
    with pytest.raises(sv.SVError):
        st.apply(np.eye(4), [2, 2])         # duplicate targets
    with pytest.raises(sv.SVError):
        st.apply(np.eye(2), [1], [n + 1])   # control out of range
    with pytest.raises(sv.SVError):
        st.set_basis(1 << n)
    np.testing.assert_array_equal(st.numpy(), before)


def test_alloc_beyond_device_memory_is_enomem():
    """A 36-qubit complex64 register (512 GiB) exceeds the device: sv_alloc
    returns SV_ENOMEM before allocating anything, and the device stays usable."""
    import ctypes
    from paper_1805_00988_amd import _lib
    lib = _lib.load()
    free0, _ = torch.cuda.mem_get_info()
    h = ctypes.c_void_p()
    rc = lib.sv_alloc(36, sv.SV_C64, None, None, ctypes.byref(h))
    assert rc == -2, rc  # SV_ENOMEM
    assert not h.value
    assert "memory" in lib.sv_last_error().decode().lower()
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free0) < (64 << 20)
    st = sv.State(10, "c64")
    assert abs(st.probabilities() - 1.0) < 1e-6
