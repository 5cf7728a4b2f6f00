"""Shared test helpers: tolerances, fidelity and GPU/oracle plumbing.

Tolerances (derived from the arithmetic):
* complex128 states: max |psi - psi_ref| <= 1e-12 (the stated target).  A
  gate rounds each output once per fused multiply-add, relative error
  <= 4 eps64 of the pair's magnitude; unitary gates do not amplify earlier
  errors, so after G gates ||delta||_2 <= 4 sqrt(2) eps64 G, i.e. 6.3e-13
  at G = 1000: 1e-12 holds with margin for every case here.
* complex64 states: the same argument with eps32 = 2^-24 gives
  ||delta||_2 <= 4 sqrt(2) eps32 G (matrix entries rounded to FP32 are
  included in the 4 ulps); element-wise checks use that bound, and every
  run also checks the fidelity target 1 - F <= 1e-6.
"""

from __future__ import annotations

import math

import numpy as np

EPS32 = 2.0 ** -24
EPS64 = 2.0 ** -53
C128_ATOL = 1e-12


def c64_bound(n_gates: int) -> float:
    return 4.0 * math.sqrt(2.0) * EPS32 * max(1, n_gates)


def fidelity(a: np.ndarray, b: np.ndarray) -> float:
    a = a.astype(np.complex128)
    b = b.astype(np.complex128)
    num = abs(np.vdot(a, b)) ** 2
    return float(num / (np.vdot(a, a).real * np.vdot(b, b).real))


def random_state(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return psi / np.linalg.norm(psi)


def assert_state_close(got: np.ndarray, ref: np.ndarray, dtype: str, n_gates: int):
    got = got.astype(np.complex128)
    err = float(np.max(np.abs(got - ref))) if got.size else 0.0
    if dtype == "c128":
        assert err <= C128_ATOL, f"max abs error {err:.3e} > {C128_ATOL:.1e}"
    else:
        bound = c64_bound(n_gates)
        assert err <= bound, f"max abs error {err:.3e} > {bound:.3e}"
        assert 1.0 - fidelity(got, ref) <= 1e-6
    return err
