"""Every HIP kernel of libsv.so keeps its working set in registers and LDS:
no private (scratch) memory, which would turn register arrays into slow
per-lane memory traffic.  Reads the resource report the build writes."""

import json
import os

import pytest

from conftest import ROOT

REPORT = os.path.join(ROOT, "paper_1805_00988_amd", "_build", "kernel_resources.json")


def test_no_kernel_uses_scratch():
    if not os.path.exists(REPORT):
        pytest.skip("library not built in this tree (run __graft_entry__.build())")
    res = json.load(open(REPORT))
    assert len(res) >= 20
    scratch = {k: v["ScratchSize"] for k, v in res.items() if v.get("ScratchSize", 0)}
    assert not scratch, scratch


def test_hot_kernels_fit_two_workgroups_per_cu():
    """Tile-pass kernels used at full size need <= 128 VGPRs so that two
    512-thread workgroups share a CU."""
    if not os.path.exists(REPORT):
        pytest.skip("library not built in this tree")
    res = json.load(open(REPORT))
    for name, v in res.items():
        if name.startswith("_ZN2sv6k_tileIfLi4E") or name.startswith("_ZN2sv6k_tileIdLi3E"):
            assert v["VGPRs"] + v.get("AGPRs", 0) <= 128, (name, v)
