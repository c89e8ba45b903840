"""torch.autograd.Function whose backward is the library's adjoint sweep.

The paper's devices give the machine-learning frameworks a custom
vector-Jacobian product so that a circuit is a black box "parameters in,
results out" (Sec. 2).  Here ``QuantumExpval`` does the same for PyTorch:

* forward: reset a device state to |0..0>, apply the gates with the given
  parameters, return <H_o> for every observable (float64 tensor);
* backward: one adjoint sweep with lambda = sum_o g_o H_o psi (the incoming
  gradient g as cotangent), which un-applies the gates from the saved final
  state instead of storing intermediate states.

All arithmetic runs in the HIP library; torch provides the device memory for
the state and the stream.
"""
from __future__ import annotations

import numpy as np
import torch

from . import qsv


class Circuit:
    """A fixed gate list and observable set on n qubits, evaluated on one GPU.

    params enter as a 1-D float64 torch tensor; ``Circuit(params)`` returns a
    float64 tensor of expectation values differentiable w.r.t. params."""

    def __init__(self, n_qubits: int, ops, observables, dtype: int = qsv.C128, device: int = 0):
        self.n = n_qubits
        self.ops = list(ops)
        self.observables = list(observables)
        self.dtype = dtype
        self.device = torch.device("cuda", device)
        self.ctx = qsv.Context(device, torch.cuda.current_stream(self.device).cuda_stream)
        self.m_obs = qsv.MarshalledObs(self.observables)
        self.tdtype = torch.complex128 if dtype == qsv.C128 else torch.complex64

    def _stream(self):
        self.ctx.set_stream(torch.cuda.current_stream(self.device).cuda_stream)

    def forward_state(self, params: np.ndarray):
        """Final state tensor and its library handle for the given params."""
        self._stream()
        t = torch.empty(1 << self.n, dtype=self.tdtype, device=self.device)
        st = qsv.State(self.ctx, self.n, self.dtype, tensor=t)
        st.reset(0)
        qsv.apply(st, self.ops, params)
        return t, st

    def __call__(self, params: torch.Tensor) -> torch.Tensor:
        return QuantumExpval.apply(params, self)


class QuantumExpval(torch.autograd.Function):
    @staticmethod
    def forward(fctx, params: torch.Tensor, circ: Circuit):
        p = params.detach().to("cpu", torch.float64).numpy().copy()
        t, st = circ.forward_state(p)
        ev = qsv.expval(st, circ.observables, marshalled=circ.m_obs)
        fctx.circ = circ
        fctx.state = st          # keeps the final-state tensor alive for backward
        fctx.params = p
        fctx.in_device = params.device
        return torch.as_tensor(ev, dtype=torch.float64, device=params.device)

    @staticmethod
    def backward(fctx, grad_out: torch.Tensor):
        circ = fctx.circ
        circ._stream()
        cot = grad_out.detach().to("cpu", torch.float64).numpy()
        grad, _ = qsv.adjoint_vjp(fctx.state, circ.ops, fctx.params, circ.observables, cot,
                                  want_expval=False, marshalled_obs=circ.m_obs)
        return torch.as_tensor(grad, dtype=torch.float64, device=fctx.in_device), None
