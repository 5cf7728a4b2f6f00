"""Host-side checks of the C-ABI library (no GPU needed): the shared library
loads, exports every entry point that include/sv.h declares, its struct
layout matches the binding, and host validation rejects bad arguments
before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT, read_golden

import paper_1805_00988_amd as sv
from paper_1805_00988_amd import _lib

HEADER = os.path.join(ROOT, "include", "sv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsv.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "sv_apply_gate" in names and "sv_adjoint_grad" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in sv.h but not exported"
    assert set(names) == set(_lib.EXPORTED)


def test_sv_op_layout():
    # int32 kind, n_targets, targets[2]; uint64 ctrl; int32 param, reserved;
    # double theta; double matrix[32]
    assert ctypes.sizeof(_lib.sv_op) == 4 * 4 + 8 + 4 * 2 + 8 + 8 * 32
    assert _lib.sv_op.ctrl_mask.offset == 16
    assert _lib.sv_op.theta.offset == 32
    assert _lib.sv_op.matrix.offset == 40


def test_state_bytes_matches_paper_memory_table(lib):
    for row in read_golden("state_memory.txt"):
        n, exact = int(row[0]), int(row[3])
        assert lib.sv_state_bytes(n, _lib.SV_C64) == exact
        assert lib.sv_state_bytes(n, _lib.SV_C128) == 2 * exact
    assert lib.sv_state_bytes(0, _lib.SV_C64) == 0
    assert lib.sv_state_bytes(41, _lib.SV_C64) == 0
    assert lib.sv_state_bytes(10, 7) == 0


def test_null_handle_and_bad_arguments_rejected(lib):
    U = np.eye(2, dtype=np.complex128).view(np.float64).reshape(-1).copy()
    t = np.array([0], np.int32)
    rc = lib.sv_apply_gate(None, 1, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), 0,
                           U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == _lib.SV_EINVAL
    assert b"NULL" in lib.sv_last_error()
    h = ctypes.c_void_p()
    assert lib.sv_alloc(0, _lib.SV_C64, None, None, ctypes.byref(h)) == _lib.SV_EINVAL
    assert lib.sv_alloc(41, _lib.SV_C64, None, None, ctypes.byref(h)) == _lib.SV_EINVAL
    assert lib.sv_alloc(10, 9, None, None, ctypes.byref(h)) == _lib.SV_EINVAL
    assert lib.sv_alloc(10, _lib.SV_C64, ctypes.c_void_p(8), None, ctypes.byref(h)) == _lib.SV_EINVAL
    assert lib.sv_free(None) == _lib.SV_EINVAL
    assert lib.sv_sync(None) == _lib.SV_EINVAL


def test_version_string(lib):
    assert lib.sv_version().startswith(b"svsim")
