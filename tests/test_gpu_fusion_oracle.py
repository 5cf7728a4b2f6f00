"""The precision/fusion workload at full size against the FP64 oracle: a
seeded 30-qubit random circuit of depth 40 (a random one-qubit gate per
qubit and 15 CZ on random pairs per layer, 1800 gates) from |0...0>.

The oracle runs the whole circuit on the host (complex128, 16 GiB of host
memory), advanced in stages of 360 gates, one test each, so that every
stage reports when it ends (tens of seconds per stage on 16 host threads).
Every variant then runs on the GPU and its final state is compared with
the oracle's over all 2^30 amplitudes:

* plain tile passes, complex128: max |psi - psi_ref| <= 1e-12;
* fused blocks of at most 4 qubits on the FP64 matrix cores, complex128:
  max |psi - psi_ref| <= 1e-12;
* plain tile passes, complex64, and fused blocks of at most 4 or 5 qubits
  with FP32 or split-BF16 matrix-core products (FP32 accumulate):
  1 - F <= 1e-6, with F = |<ref|psi>|^2 / (|ref|^2 |psi|^2) in FP64 and the
  maximum amplitude error reported beside it.
"""

import math

import numpy as np
import pytest

import circuits as C
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1805_00988_amd as sv  # noqa: E402

O.build(force=False)

N = 30
STAGES = 5


@pytest.fixture(scope="module")
def workload():
    circ = C.config2(n=N, seed=0, depth=40)
    w = {"circ": circ, "psi": None, "done": 0}
    yield w
    w["psi"] = None  # release the 16 GiB oracle state before the next module


def advance(w, stage):
    """Run the oracle up to the end of the given stage (0-based)."""
    gates = w["circ"].gates
    per = math.ceil(len(gates) / STAGES)
    if w["psi"] is None:
        w["psi"] = O.basis_state(N, 0)
        w["done"] = 0
    while w["done"] <= stage:
        s = w["done"]
        O.run_gates(N, gates[s * per:(s + 1) * per], w["psi"])
        w["done"] = s + 1


def compare(st, ref):
    """(1 - F, max |psi - ref|) over all amplitudes, chunk by chunk in FP64."""
    ov, na, nr, mx = 0j, 0.0, 0.0, 0.0
    step = 1 << 26
    for c0 in range(0, ref.size, step):
        got = st.amps[c0:c0 + step].cpu().numpy().astype(np.complex128)
        r = ref[c0:c0 + step]
        ov += np.vdot(r, got)
        na += float(np.vdot(got, got).real)
        nr += float(np.vdot(r, r).real)
        mx = max(mx, float(np.max(np.abs(got - r))))
    return 1.0 - abs(ov) ** 2 / (na * nr), mx


@pytest.mark.parametrize("stage", range(STAGES))
def test_oracle_stage(workload, stage):
    advance(workload, stage)
    assert workload["done"] == stage + 1
    if stage == STAGES - 1:
        # the oracle's own invariant: unit norm after the whole circuit
        assert abs(float(np.vdot(workload["psi"], workload["psi"]).real) - 1.0) < 1e-12


VARIANTS = [
    # label, dtype, k_max (0 = plain tile passes), prec
    ("plain_c128", "c128", 0, sv.SV_PREC_NATIVE),
    ("fused_k4_fp64", "c128", 4, sv.SV_PREC_NATIVE),
    ("plain_c64", "c64", 0, sv.SV_PREC_NATIVE),
    ("fused_k4_fp32", "c64", 4, sv.SV_PREC_FP32),
    ("fused_k5_fp32", "c64", 5, sv.SV_PREC_FP32),
    ("fused_k4_bf16x3", "c64", 4, sv.SV_PREC_SPLIT_BF16),
    ("fused_k5_bf16x3", "c64", 5, sv.SV_PREC_SPLIT_BF16),
]


@pytest.mark.parametrize("label,dtype,k,prec", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_fusion_workload_vs_oracle(workload, label, dtype, k, prec):
    advance(workload, STAGES - 1)
    circ = workload["circ"]
    st = sv.State(N, dtype)
    if k == 0:
        st.run(circ.gates, mode=sv.SV_RUN_TILED)
        blocks = None
    else:
        blocks = st.run_fused(circ.gates, k_max=k, prec=prec)
    infid, mx = compare(st, workload["psi"])
    print(f"{label}: blocks={blocks} 1-F={infid:.3e} max|err|={mx:.3e}", flush=True)
    if dtype == "c128":
        assert mx <= 1e-12, (label, mx)
    assert infid <= 1e-6, (label, infid)
    del st
    torch.cuda.empty_cache()
