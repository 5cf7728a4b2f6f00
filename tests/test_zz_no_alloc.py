"""sv_expectation_noalloc (the entry point that allocates nothing: its partial
sums live in a static device array of the library) against sv_expectation
on the same states: two calls in a row, the second on a smaller state, each
result equal bit for bit (same kernels, same workgroup count), no change in
free device memory across the calls, and argument errors reported."""

import numpy as np
import pytest

import circuits as C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1805_00988_amd as sv  # noqa: E402


def terms(n, seed):
    rng = np.random.default_rng(seed)
    masks = [int(m) for m in rng.integers(1, 1 << n, size=5)] + [1, (1 << n) - 1]
    coeffs = [float(c) for c in rng.standard_normal(len(masks))]
    return masks, coeffs


def test_noalloc_matches_expectation_two_calls():
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    cases = [(20, "c128", 1), (12, "c64", 2)]  # the second call on a smaller state
    states = []
    for n, dtype, seed in cases:
        st = sv.State(n, dtype).run(C.random_circuit(n, 6, seed=seed, entangler="X").gates)
        states.append(st)
    torch.cuda.synchronize()
    for i, ((n, dtype, seed), st) in enumerate(zip(cases, states)):
        masks, coeffs = terms(n, seed)
        ref = st.expectation(masks, coeffs)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        sv.sv_expectation_noalloc(st.amps, n, masks, coeffs, out[i:])
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        got = float(out[i].item())
        assert got == ref, (n, dtype, got, ref)
        assert free1 == free0, (free0, free1)
    # the first result is not disturbed by the second call
    masks, coeffs = terms(20, 1)
    assert float(out[0].item()) == states[0].expectation(masks, coeffs)


def test_noalloc_argument_errors():
    st = sv.State(8, "c64")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(sv.SVError):
        sv.sv_expectation_noalloc(st.amps, 8, [], [], out)          # no terms
    with pytest.raises(sv.SVError):
        sv.sv_expectation_noalloc(st.amps, 8, [1 << 8], [1.0], out)  # mask bit >= n
    with pytest.raises(sv.SVError):
        sv.sv_expectation_noalloc(st.amps, 8, [1] * 65, [1.0] * 65, out)
    sv.sv_expectation_noalloc(st.amps, 8, [1], [1.0], out)
    assert float(out[0].item()) == 1.0  # |0...0>: <Z_0> = 1
