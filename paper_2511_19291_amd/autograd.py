"""torch.autograd.Function over the adjoint backward (the paper's invertible
execution, Sec. 4.4 and the `invertible=True` device of Appendix A).

Forward: reset the state to |0..0>, run the circuit with the given
parameters, return L = sum_t coeff_t <P_t> per batch row. Once
2n + log2(batch) >= 44 (``fuse``: batch 16 from 20 qubits, batch 1 from 22),
the gates are fused into 5-qubit blocks on the matrix cores (Sec. 4.1.1);
runs of per-row gates (an input encoding) with one matrix per row. Backward: the library un-applies the gates from the forward output
(x = U^* y) and accumulates dL/dtheta in FP64; nothing is stored between the
passes except the final state itself. By default the backward groups the
gates into 4-qubit blocks on the matrix cores (``sv_adjoint_grad_mfma``, one
sweep per block) from 13 qubits when every gate fits; ``block_qubits=0``
selects the per-gate backward, 3..5 the VALU blocks. The state object
therefore holds one pending forward at a time: run backward before the next
forward on the same state. Every backward checks this: it raises
``StaleStateError`` when the state changed after the forward that saved it
(a second forward on the same state, or a second backward through the same
graph, whose first backward has already un-applied the gates), and when the
recomputed start state drifts from |0..0> by more than ``DRIFT_MAX``.
"""

from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import torch

from . import sv


class StaleStateError(RuntimeError):
    """The state no longer holds the forward output a backward needs."""


# Largest accepted distance ||psi_recomputed - |0..0>|| after the backward has
# un-applied every gate (Sec. 4.4: the layer inputs are recomputed from the
# output, so the recomputed start state must be the true one). Complex64
# rounding of the forward and of the un-apply grows like sqrt(G) 2^-24 per
# sweep, about 1e-4 for 10^6 gates; a state that is not the forward's output
# is off by O(1).
DRIFT_MAX = 1e-3


def _saved_version(ctx, state) -> None:
    ctx.state = state
    ctx.version = state.version


def _check_fresh(ctx) -> None:
    if ctx.state.version != ctx.version:
        raise StaleStateError(
            "the state changed after this forward (another forward on the same state, or a second "
            "backward through the same graph): the adjoint backward needs the forward's output state")


def _check_drift(drift) -> None:
    d = float(np.max(drift)) if np.size(drift) else 0.0
    if not d <= DRIFT_MAX:
        raise StaleStateError(f"recomputed start state drifts by {d:.3e} (> {DRIFT_MAX:.0e}): "
                              "the backward did not start from this forward's output")


# The forward fuses the gates into matrix-core blocks once the state is
# large enough for the blocks to repay their host planning: measured on one
# MI355X, batch 16 from 20 qubits (18: 1.9 ms per-gate vs 2.8 ms fused; 20:
# 5.9 vs 4.5) and batch 1 from 22 (20: 2.8 vs 3.9 ms; 22: 6.5 vs 5.1), i.e.
# 2n + log2(batch) >= 44.
FUSED_FORWARD_MIN_QUBITS = 20


def default_fuse(circuit, batch: int = 1) -> bool:
    return 2 * circuit.n + np.log2(max(int(batch), 1)) >= 2 * FUSED_FORWARD_MIN_QUBITS + 4


def _forward(state, circuit, p, fuse: bool) -> None:
    state.reset()
    if fuse:
        state.run_fused(circuit, params=p)
    else:
        state.run(circuit, params=p)


# Backward form by width (measured on one MI355X, rings and batched ladders of
# 10 to 28 qubits): below 13 qubits the per-gate backward (launch-bound
# sizes), from 13 the matrix-core blocks, which from there on match or beat
# both the per-gate and the 4-qubit VALU blocked backward. The VALU blocks stay
# available through ``block_qubits``.
MFMA_MIN_QUBITS = 13


def default_block_qubits(circuit) -> int:
    """Backward form for this circuit: ``sv.ADJOINT_MFMA`` (matrix-core
    blocks) from 13 qubits when every gate fits in four qubits, else 0 (per
    gate)."""
    fits = all(len(op.targets) + len(op.controls) <= 4 for op in circuit.ops)
    if fits and circuit.n >= MFMA_MIN_QUBITS:
        return sv.ADJOINT_MFMA
    return 0


class AdjointExpval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, circuit, terms: Sequence[Tuple[float, int, int]], state: "sv.State",
                block_qubits: int = 0, fuse: bool = False):
        ctx.block_qubits = block_qubits
        p = np.ascontiguousarray(params.detach().to("cpu", torch.float64).numpy())
        _forward(state, circuit, p, fuse)
        vals = state.expval(terms)                 # [batch, n_terms]
        loss = vals.sum(axis=1)
        ctx.circuit = circuit
        ctx.terms = list(terms)
        _saved_version(ctx, state)
        ctx.p = p
        ctx.shape = params.shape
        out = torch.from_numpy(loss).to(device=params.device, dtype=params.dtype)
        return out if params.dim() == 2 else out.reshape(())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        _check_fresh(ctx)
        _, grad, drift = ctx.state.adjoint_grad(ctx.circuit, ctx.terms, params=ctx.p, block_qubits=ctx.block_qubits)
        _check_drift(drift)
        go = grad_out.detach().to("cpu", torch.float64).reshape(-1, 1).numpy()
        g = grad * go                              # [batch, n_params]
        g = torch.from_numpy(g.reshape(ctx.shape)).to(device=grad_out.device, dtype=grad_out.dtype)
        return g, None, None, None, None, None


class QuantumExpval(torch.nn.Module):
    """A fixed circuit and observable; forward(params) -> L (per batch row),
    differentiable through the adjoint backward."""

    def __init__(self, circuit, terms: Sequence[Tuple[float, int, int]], batch: int = 1, device=None,
                 block_qubits=None, fuse=None):
        super().__init__()
        self.circuit = circuit
        self.terms = list(terms)
        self.state = sv.State(circuit.n, batch, device=device)
        self.block_qubits = default_block_qubits(circuit) if block_qubits is None else block_qubits
        self.fuse = default_fuse(circuit, batch) if fuse is None else bool(fuse)

    def forward(self, params: torch.Tensor) -> torch.Tensor:
        return AdjointExpval.apply(params, self.circuit, self.terms, self.state, self.block_qubits, self.fuse)


class ExpvalZ(torch.autograd.Function):
    """<Z_i> of every qubit for every batch row, differentiable in the rows'
    parameters (inputs and angles alike). Backward: with g = dF/d<Z_i>_r from
    the upstream graph, the library's adjoint runs once for all rows with the
    observable sum_i g[r, i] Z_i of row r (``sv_adjoint_grad_weighted``)."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, circuit, state: "sv.State", block_qubits: int = 0, fuse: bool = False):
        ctx.block_qubits = block_qubits
        p = np.ascontiguousarray(params.detach().to("cpu", torch.float64).numpy().reshape(state.batch, circuit.n_params))
        _forward(state, circuit, p if state.batch > 1 else p[0], fuse)
        z = state.expval_z_all()[:, : circuit.n]
        ctx.circuit = circuit
        _saved_version(ctx, state)
        ctx.p = p
        ctx.shape = params.shape
        return torch.from_numpy(np.ascontiguousarray(z)).to(device=params.device, dtype=params.dtype)

    @staticmethod
    def backward(ctx, grad_z: torch.Tensor):
        n = ctx.circuit.n
        terms = [(1.0, 0, 1 << i) for i in range(n)]
        g = np.ascontiguousarray(grad_z.detach().to("cpu", torch.float64).numpy().reshape(ctx.state.batch, n))
        p = ctx.p if ctx.state.batch > 1 else ctx.p[0]
        _check_fresh(ctx)
        _, grad, drift = ctx.state.adjoint_grad(ctx.circuit, terms, params=p, coeff_rows=g,
                                                block_qubits=ctx.block_qubits)
        _check_drift(drift)
        out = torch.from_numpy(grad.reshape(ctx.shape)).to(device=grad_z.device, dtype=grad_z.dtype)
        return out, None, None, None, None


class MeasureAllZ(torch.nn.Module):
    """A fixed circuit on a batch of states; forward(params [batch, P]) ->
    [batch, n] of <Z_i> (exact, shots = 0), differentiable through the
    adjoint backward (the appendix example's measure_allZ on an invertible
    device)."""

    def __init__(self, circuit, batch: int = 1, device=None, block_qubits=None, fuse=None):
        super().__init__()
        self.circuit = circuit
        self.state = sv.State(circuit.n, batch, device=device)
        self.block_qubits = default_block_qubits(circuit) if block_qubits is None else block_qubits
        self.fuse = default_fuse(circuit, batch) if fuse is None else bool(fuse)

    def forward(self, params: torch.Tensor) -> torch.Tensor:
        return ExpvalZ.apply(params, self.circuit, self.state, self.block_qubits, self.fuse)


class GaussianExpvalZ(torch.autograd.Function):
    """Shot-noise estimates of every <Z_i> (Sec. 4.3.2's Gaussian limit of the
    multinomial), differentiable by reparameterisation: for fixed normals z
    the estimate is a smooth function of the probabilities, so its backward
    is the adjoint (Sec. 4.4) started from the diagonal observable
    w_b = dF/d|psi_b|^2 that the library derives from the upstream gradient.
    ``normals``: device float64 [batch, 2^n] (drawn by the caller)."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, circuit, state: "sv.State", normals: torch.Tensor, shots: float,
                block_qubits: int = 0, fuse: bool = False):
        p = np.ascontiguousarray(params.detach().to("cpu", torch.float64).numpy().reshape(state.batch, circuit.n_params))
        _forward(state, circuit, p if state.batch > 1 else p[0], fuse)
        est = np.stack([state.gaussian_expval_z(normals[r], shots, row=r) for r in range(state.batch)])
        ctx.circuit, ctx.p, ctx.shape = circuit, p, params.shape
        _saved_version(ctx, state)
        ctx.normals, ctx.shots, ctx.block_qubits = normals, shots, block_qubits
        return torch.from_numpy(est).to(device=params.device, dtype=params.dtype)

    @staticmethod
    def backward(ctx, grad_e: torch.Tensor):
        _check_fresh(ctx)
        st = ctx.state
        g = np.ascontiguousarray(grad_e.detach().to("cpu", torch.float64).numpy().reshape(st.batch, ctx.circuit.n))
        w = torch.empty((st.batch, 1 << st.n), dtype=torch.float64, device=st.tensor.device)
        for r in range(st.batch):
            st.gaussian_expval_z_backward(ctx.normals[r], ctx.shots, g[r], row=r, out=w[r])
        p = ctx.p if st.batch > 1 else ctx.p[0]
        _, grad, drift = st.adjoint_grad_diag(ctx.circuit, w, params=p, block_qubits=ctx.block_qubits)
        _check_drift(drift)
        out = torch.from_numpy(grad.reshape(ctx.shape)).to(device=grad_e.device, dtype=grad_e.dtype)
        return out, None, None, None, None, None, None
