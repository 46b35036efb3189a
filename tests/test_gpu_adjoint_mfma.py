"""GPU parity of the matrix-core blocked backward (sv_adjoint_grad_mfma):
per 4-qubit block, one sweep computes the block's correlation
S = sum_c psi_c lambda_c^* on FP64 matrix cores and un-applies the block's
product on FP32 matrix cores; each derivative is 2 Re Tr(X_k S) with X_k
formed on the host in FP64, or, for blocks whose parameters differ between
rows and for batches of at most four rows, Tr(G_k S_t) with S stepped down
the block's gates on the host (S_t = W_t^* S W_t).

References: the oracle's FP64 adjoint (pinned against parameter shift and
central differences) and parameter shift itself, relative 1e-4 (2-norm and
per component) as for the other backward forms; the per-gate GPU backward on
the same state (relative 2e-5). S's products of FP32 data are exact in FP64,
so the derivatives carry only the complex64 state's own rounding."""

import numpy as np
import pytest
import torch

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod

pytestmark = pytest.mark.gpu

REL = 1e-4
MF = svmod.ADJOINT_MFMA


def _close(g, ref, rel=REL):
    scale = max(np.linalg.norm(ref), 1e-12)
    assert np.linalg.norm(g - ref) / scale <= rel, np.linalg.norm(g - ref) / scale
    assert np.max(np.abs(g - ref)) <= rel * max(np.max(np.abs(ref)), 1e-12)


def test_ring14_vs_parameter_shift(sv):
    circ = C.WORKLOADS["ring14"]()
    terms = C.z_sum_terms(14)
    st = sv.State(14).reset().run(circ)
    loss, g, drift = st.adjoint_grad(circ, terms, block_qubits=MF)
    _close(g[0], oracle.grad_param_shift(circ, terms))
    assert abs(loss[0] - oracle.loss(circ, terms)) < 1e-4
    assert drift[0] < 1e-4
    assert abs(st.to_numpy()[0][0] - 1) < 1e-4


@pytest.mark.parametrize("n,seed", [(9, 2), (10, 5), (12, 3)])
def test_every_kind_vs_oracle_adjoint(sv, n, seed):
    """Random circuits of every kind (controls, two-target kinds, U3 with
    three parameters, phase gates, up to two controls) and observables with X
    and Y strings (a complex co-state)."""
    circ = C.random_circuit(n, 90, 60 + seed, max_controls=2)
    rng = np.random.default_rng(seed)
    terms = [(float(rng.normal()), int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n))) for _ in range(4)]
    st = sv.State(n).reset().run(circ)
    loss, g, drift = st.adjoint_grad(circ, terms, block_qubits=MF)
    ref_loss, ref, _ = oracle.grad_adjoint(circ, terms)
    _close(g[0], ref)
    assert abs(loss[0] - ref_loss) < 1e-4
    assert drift[0] < 1e-4


def test_matches_per_gate_backward(sv):
    circ = C.rxry_ring(16, 4, 9)
    terms = C.z_sum_terms(16)
    st = sv.State(16)
    st.reset().run(circ)
    _, g_gate, _ = st.adjoint_grad(circ, terms)
    st.reset().run(circ)
    _, g_m, d = st.adjoint_grad(circ, terms, block_qubits=MF)
    _close(g_m[0], g_gate[0], rel=2e-5)
    assert d[0] < 1e-4


def test_batched_rows_weighted(sv):
    """Per-row inputs (per-row block products inside one launch) and
    per-row observable weights."""
    n, B = 10, 4
    circ, rows = C.profiling_ladder(n, 3, B, seed=12)
    coeff = np.random.default_rng(13).normal(size=(B, n))
    terms = [(1.0, 0, 1 << i) for i in range(n)]
    st = sv.State(n, B)
    st.reset().run(circ, params=rows)
    loss, g, drift = st.adjoint_grad(circ, terms, params=rows, coeff_rows=coeff, block_qubits=MF)
    for r in range(B):
        wt = [(float(coeff[r, i]), 0, 1 << i) for i in range(n)]
        ref_loss, ref, _ = oracle.grad_adjoint(circ, wt, params=rows[r])
        _close(g[r], ref)
        assert abs(loss[r] - ref_loss) < 1e-4
    assert np.all(drift < 1e-4)


def test_batched_shared_and_per_row_blocks(sv):
    """Batch 6 (more rows than the host's S recursion takes for shared
    blocks): the shared ansatz blocks take their derivatives from X_k formed
    on the host, the per-row encoding blocks from the S recursion, in one
    chunked pipeline; every row against the oracle's adjoint."""
    n, B = 11, 6
    circ, rows = C.profiling_ladder(n, 3, B, seed=21)
    coeff = np.random.default_rng(22).normal(size=(B, n))
    terms = [(1.0, 0, 1 << i) for i in range(n)]
    st = sv.State(n, B)
    st.reset().run(circ, params=rows)
    loss, g, drift = st.adjoint_grad(circ, terms, params=rows, coeff_rows=coeff, block_qubits=MF)
    for r in range(B):
        wt = [(float(coeff[r, i]), 0, 1 << i) for i in range(n)]
        ref_loss, ref, _ = oracle.grad_adjoint(circ, wt, params=rows[r])
        _close(g[r], ref)
        assert abs(loss[r] - ref_loss) < 1e-4
    assert np.all(drift < 1e-4)


def test_diagonal_observable(sv):
    """sv_adjoint_grad_diag with the matrix-core backward equals its Pauli
    form for W = diag(sum_i s_i)."""
    n = 11
    circ = C.rxry_ring(n, 2, 4)
    st = sv.State(n)
    st.reset().run(circ)
    _, g_p, _ = st.adjoint_grad(circ, C.z_sum_terms(n))
    b = np.arange(1 << n)
    w = sum(1.0 - 2.0 * ((b >> i) & 1) for i in range(n)).astype(np.float64)
    st.reset().run(circ)
    _, g_d, drift = st.adjoint_grad_diag(circ, torch.tensor(w, device="cuda").reshape(1, -1).contiguous(),
                                         block_qubits=MF)
    _close(g_d[0], g_p[0], rel=2e-5)
    assert drift[0] < 1e-4


def test_paper_size_vs_per_gate(sv):
    """22 qubits, 10 layers: the matrix-core backward against the per-gate
    GPU backward on the same forward state."""
    circ = C.rxry_ring(22, 6, 17)
    terms = C.z_sum_terms(22)
    st = sv.State(22)
    st.reset().run(circ)
    _, g_gate, _ = st.adjoint_grad(circ, terms)
    st.reset().run(circ)
    _, g_m, d = st.adjoint_grad(circ, terms, block_qubits=MF)
    _close(g_m[0], g_gate[0], rel=2e-5)
    assert d[0] < 1e-4
    st.free()


def test_many_rows_more_groups_per_wave(sv):
    """520 rows of 20 qubits: four groups of 512 amplitudes per wave would
    need more than 2^16 workgroups for the launch's parts of S, so each wave
    takes eight groups (a different tiling of the same sweep). Every row
    against the per-gate GPU backward; rows 0 and 519 also against a 10-row
    run of the same inputs, which takes four groups per wave."""
    n, B = 20, 520
    circ, rows = C.profiling_ladder(n, 1, B, seed=31)
    terms = C.z_sum_terms(n)
    st = sv.State(n, B)
    st.reset().run(circ, params=rows)
    _, g_gate, _ = st.adjoint_grad(circ, terms, params=rows)
    st.reset().run(circ, params=rows)
    _, g_m, d = st.adjoint_grad(circ, terms, params=rows, block_qubits=MF)
    for r in range(B):
        _close(g_m[r], g_gate[r], rel=2e-5)
    assert np.all(d < 1e-4)
    st.free()
    sub = np.ascontiguousarray(rows[[0, B - 1] * 5])
    s2 = sv.State(n, 10)
    s2.reset().run(circ, params=sub)
    _, g_s, _ = s2.adjoint_grad(circ, terms, params=sub, block_qubits=MF)
    _close(g_s[0], g_m[0], rel=2e-5)
    _close(g_s[1], g_m[B - 1], rel=2e-5)
    s2.free()


def test_refusals(sv):
    st = sv.State(8).reset()
    with pytest.raises(svmod.SvError) as e:
        st.adjoint_grad(C.ghz(8), C.z_sum_terms(8), block_qubits=MF)
    assert e.value.status == 4
    b = C._Builder(10)
    b.gate("rxx", [0, 1], [2, 3, 4], values=[0.3])
    wide = b.build("wide_gate")
    st10 = sv.State(10).reset().run(wide)
    with pytest.raises(svmod.SvError) as e:
        st10.adjoint_grad(wide, C.z_sum_terms(10), block_qubits=MF)
    assert e.value.status == 4
