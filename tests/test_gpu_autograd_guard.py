"""The autograd layers refuse a backward that would un-apply the gates from a
state other than their forward's output (Sec. 4.4 recomputes each layer input
as x = U^* y from that output, so any other starting state gives silently
wrong gradients):

* a second forward on the same state before the first forward's backward;
* a second backward through the same graph (retain_graph=True): the first
  backward already took the state back to |0..0>;
* a state changed behind the library's back (a write through the tensor),
  caught by the drift of the recomputed start state.

Each layer (AdjointExpval, ExpvalZ, GaussianExpvalZ) and each backward form
is covered; a plain forward/backward still matches the oracle.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod
from paper_2511_19291_amd.autograd import (GaussianExpvalZ, MeasureAllZ, QuantumExpval,
                                           StaleStateError)

pytestmark = pytest.mark.gpu

FORMS = [0, 4, svmod.ADJOINT_MFMA]
FORM_IDS = ["per_gate", "valu_blocks", "mfma_blocks"]


@pytest.mark.parametrize("bq", FORMS, ids=FORM_IDS)
def test_two_forwards_then_backward_raises(sv, bq):
    circ = C.rxry_ring(9, 2, 3)           # the matrix-core form needs >= 9 qubits
    mod = QuantumExpval(circ, C.z_sum_terms(9), block_qubits=bq)
    a = torch.tensor(circ.params, requires_grad=True)
    b = torch.tensor(circ.params + 0.1, requires_grad=True)
    la = mod(a)
    lb = mod(b)                       # overwrites the state la's backward needs
    with pytest.raises(StaleStateError):
        la.backward()
    lb.backward()                     # the latest forward is still fine
    ref = oracle.grad_param_shift(circ, C.z_sum_terms(9), params=circ.params + 0.1)
    np.testing.assert_allclose(b.grad.numpy(), ref, atol=1e-4 * np.max(np.abs(ref)))


@pytest.mark.parametrize("bq", FORMS, ids=FORM_IDS)
def test_retain_graph_second_backward_raises(sv, bq):
    circ, rows = C.profiling_ladder(9, 2, 3, seed=5)
    layer = MeasureAllZ(circ, 3, block_qubits=bq)
    x = torch.tensor(rows, requires_grad=True)
    z = layer(x)
    loss = (z * z).sum()
    loss.backward(retain_graph=True)
    g1 = x.grad.clone()
    with pytest.raises(StaleStateError):
        loss.backward()
    assert torch.equal(x.grad, g1)    # the refused backward added nothing
    for r in range(3):
        zr, _ = oracle.expval_z_all(oracle.run(circ, params=rows[r]), 9)
        want = oracle.grad_param_shift(circ, [(2.0 * zr[i], 0, 1 << i) for i in range(9)], params=rows[r])
        np.testing.assert_allclose(g1[r].numpy(), want, atol=1e-4 * np.max(np.abs(want)))


def test_state_written_behind_the_library_raises(sv):
    """A write through the tensor is not counted by the state's version;
    the recomputed start state then drifts by O(1) and the backward refuses
    it instead of returning its gradient."""
    circ = C.rxry_ring(7, 2, 9)
    mod = QuantumExpval(circ, C.z_sum_terms(7), block_qubits=0)
    th = torch.tensor(circ.params, requires_grad=True)
    loss = mod(th)
    t = mod.state.tensor
    t[0] = torch.roll(t[0], 1)        # a different (still normalised) state
    with pytest.raises(StaleStateError, match="drifts"):
        loss.backward()


def test_gaussian_layer_refuses_stale_state(sv):
    n = 6
    circ, rows = C.profiling_ladder(n, 1, 1, seed=3)
    st = svmod.State(n, 1)
    normals = torch.tensor(np.random.default_rng(4).normal(size=(1, 1 << n)), device="cuda")
    x = torch.tensor(rows[0], requires_grad=True)
    e = GaussianExpvalZ.apply(x, circ, st, normals, 1000.0, 0, False)
    st.reset()                        # another use of the state in between
    with pytest.raises(StaleStateError):
        e.sum().backward()
    x2 = torch.tensor(rows[0], requires_grad=True)
    e2 = GaussianExpvalZ.apply(x2, circ, st, normals, 1000.0, 0, False)
    e2.sum().backward()               # fresh forward: accepted
    assert torch.all(torch.isfinite(x2.grad))
