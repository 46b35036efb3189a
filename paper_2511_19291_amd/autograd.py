"""torch.autograd.Function over the adjoint backward (the paper's invertible
execution, Sec. 4.4 and the `invertible=True` device of Appendix A).

Forward: reset the state to |0..0>, run the circuit with the given
parameters, return L = sum_t coeff_t <P_t> per batch row. Backward: the
library un-applies the gates from the forward output (x = U^* y) and
accumulates dL/dtheta in FP64; nothing is stored between the passes except
the final state itself. The state object therefore holds one pending
forward at a time: run backward before the next forward on the same state.
"""

from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import torch

from . import sv


class AdjointExpval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, circuit, terms: Sequence[Tuple[float, int, int]], state: "sv.State"):
        p = np.ascontiguousarray(params.detach().to("cpu", torch.float64).numpy())
        state.reset()
        state.run(circuit, params=p)
        vals = state.expval(terms)                 # [batch, n_terms]
        loss = vals.sum(axis=1)
        ctx.circuit = circuit
        ctx.terms = list(terms)
        ctx.state = state
        ctx.p = p
        ctx.shape = params.shape
        out = torch.from_numpy(loss).to(device=params.device, dtype=params.dtype)
        return out if params.dim() == 2 else out.reshape(())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        _, grad, _ = ctx.state.adjoint_grad(ctx.circuit, ctx.terms, params=ctx.p)
        go = grad_out.detach().to("cpu", torch.float64).reshape(-1, 1).numpy()
        g = grad * go                              # [batch, n_params]
        g = torch.from_numpy(g.reshape(ctx.shape)).to(device=grad_out.device, dtype=grad_out.dtype)
        return g, None, None, None


class QuantumExpval(torch.nn.Module):
    """A fixed circuit and observable; forward(params) -> L (per batch row),
    differentiable through the adjoint backward."""

    def __init__(self, circuit, terms: Sequence[Tuple[float, int, int]], batch: int = 1, device=None):
        super().__init__()
        self.circuit = circuit
        self.terms = list(terms)
        self.state = sv.State(circuit.n, batch, device=device)

    def forward(self, params: torch.Tensor) -> torch.Tensor:
        return AdjointExpval.apply(params, self.circuit, self.terms, self.state)
