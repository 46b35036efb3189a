"""Run-to-run bit equality of the forward and backward forms.

Every reduction in the library sums in a fixed order (per-wave registers,
then fixed trees of partial sums; no floating-point atomics), and the host
side of the backward forms its derivatives from those sums in FP64 in a
fixed order, so repeating a call on the same inputs must give the same bits:
the fused forward in each matrix-core mode, every backward form (per gate,
blocked on 4 and 5 qubits, matrix-core blocks; with shared and with per-row
angles), and the start state each backward recomputes by un-applying the
circuit (Sec. 4.4)."""

import numpy as np
import pytest

from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,max_k", [(svmod.FUSED_FP32_MFMA, 5), (svmod.FUSED_BF16X3, 5),
                                        (svmod.FUSED_BF16X3, 6)])
def test_fused_forward_bitwise_repeatable(sv, mode, max_k):
    n = 18
    circ = C.brickwork_u3_cz(n, 6, 23)
    print(f"fused forward n={n} mode={mode} max_k={max_k}", flush=True)
    st = sv.State(n)
    a = st.reset().run_fused(circ, max_k=max_k, mode=mode).to_numpy()
    b = st.reset().run_fused(circ, max_k=max_k, mode=mode).to_numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    st.free()


@pytest.mark.parametrize("block", [0, 4, 5, svmod.ADJOINT_MFMA])
def test_backward_bitwise_repeatable(sv, block):
    n = 16
    circ = C.rxry_ring(n, 4, 29)
    terms = C.z_sum_terms(n)
    print(f"backward n={n} block_qubits={block}", flush=True)
    st = sv.State(n)
    out = []
    for _ in range(2):
        st.reset().run(circ)
        loss, grad, drift = st.adjoint_grad(circ, terms, block_qubits=block)
        out.append((loss, grad, drift, st.to_numpy()))
    (l0, g0, d0, s0), (l1, g1, d1, s1) = out
    assert np.array_equal(l0, l1) and np.array_equal(g0, g1) and np.array_equal(d0, d1)
    assert np.array_equal(s0.view(np.uint32), s1.view(np.uint32))
    assert np.all(np.isfinite(g0)) and np.linalg.norm(g0) > 0
    st.free()


@pytest.mark.parametrize("block", [0, svmod.ADJOINT_MFMA])
def test_batched_backward_bitwise_repeatable(sv, block):
    """Per-row input angles (the profiling ladder at batch 6): the per-gate
    and matrix-core backward, each row's gradient the same bits twice."""
    n, B = 14, 6
    circ, rows = C.profiling_ladder(n, 2, B, seed=37)
    terms = C.z_sum_terms(n)
    print(f"batched backward n={n} batch={B} block_qubits={block}", flush=True)
    st = sv.State(n, B)
    out = []
    for _ in range(2):
        st.reset().run(circ, params=rows)
        _, grad, drift = st.adjoint_grad(circ, terms, params=rows, block_qubits=block)
        out.append((grad, drift))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    st.free()
