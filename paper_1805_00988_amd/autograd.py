"""Adjoint-method gradients behind torch.autograd.Function.

``ExpectationCircuit`` owns two device registers (the state and the adjoint
work vector).  Its forward runs the parametrised circuit from |0...0> and
returns <psi|H|psi> for a Z-string observable H; backward calls the
library's adjoint sweep (sv_adjoint_grad), which returns dL/dparams for all
parameters from one reverse pass over the circuit.
"""

from __future__ import annotations

import numpy as np

from . import (SV_RUN_TILED, State, ops_from_gates, sv_adjoint_grad, sv_expectation, sv_run,
               sv_set_basis)


def _torch():
    import torch
    return torch


class ExpectationCircuit:
    def __init__(self, n_qubits: int, gates, z_masks, coeffs, dtype="c128", mode: int = SV_RUN_TILED):
        self.n = n_qubits
        self.gates = list(gates)
        self.z_masks = list(z_masks)
        self.coeffs = list(coeffs)
        self.mode = mode
        self.psi = State(n_qubits, dtype)
        self.lam = State(n_qubits, dtype)
        # parameters whose circuit output psi currently holds (None: psi does
        # not hold a circuit output)
        self._psi_params = None

    def loss(self, params) -> float:
        """<H> at the given parameters (leaves psi holding the circuit output)."""
        params = np.array(params, np.float64)  # a copy: the caller may change its array
        sv_set_basis(self.psi.handle, 0)
        sv_run(self.psi.handle, self.gates, params, self.mode)
        self._psi_params = params
        return sv_expectation(self.psi.handle, self.z_masks, self.coeffs)

    def loss_and_grad(self, params):
        """(loss, gradient) at params; the forward circuit is run again unless
        psi already holds its output for exactly these parameters."""
        params = np.asarray(params, np.float64)
        if self._psi_params is None or not np.array_equal(self._psi_params, params):
            self.loss(params)
        self._psi_params = None  # the sweep leaves psi at the input state
        return sv_adjoint_grad(self.psi.handle, self.lam.handle, self.gates, params,
                               self.z_masks, self.coeffs)

    def __call__(self, params):
        return AdjointExpectation.apply(params, self)


def _make_function():
    torch = _torch()

    class _AdjointExpectation(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, circuit):
            p = params.detach().cpu().double().numpy()
            value = circuit.loss(p)
            ctx.circuit = circuit
            ctx.params = p
            ctx.device = params.device
            return torch.tensor(value, dtype=torch.float64, device=params.device)

        @staticmethod
        def backward(ctx, grad_out):
            # loss_and_grad reruns the forward circuit when psi holds another
            # parameter vector's output (e.g. a later forward call)
            _, grad = ctx.circuit.loss_and_grad(ctx.params)
            g = torch.from_numpy(grad).to(ctx.device) * grad_out.to(torch.float64)
            return g, None

    return _AdjointExpectation


class _Lazy:
    _fn = None

    def apply(self, params, circuit):
        if _Lazy._fn is None:
            _Lazy._fn = _make_function()
        return _Lazy._fn.apply(params, circuit)


AdjointExpectation = _Lazy()
