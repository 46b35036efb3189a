"""GPU parity of the blocked adjoint backward (one sweep per block of gates
on 3, 4 or 5 qubits, gates un-applied in registers) against the oracle's exact
gradients, and against the per-gate GPU backward.

Tolerance as the per-gate adjoint: relative 1e-4 (2-norm and per
component). The Pauli-rotation derivative terms use FP32 pairwise products
with FP64 accumulation: the products carry the complex64 data's own
rounding (2^-24 relative), far inside 1e-4."""

import numpy as np
import pytest

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod

pytestmark = pytest.mark.gpu

REL = 1e-4


def _close(g, ref, rel=REL):
    scale = max(np.linalg.norm(ref), 1e-12)
    assert np.linalg.norm(g - ref) / scale <= rel, np.linalg.norm(g - ref) / scale
    assert np.max(np.abs(g - ref)) <= rel * max(np.max(np.abs(ref)), 1e-12)


@pytest.mark.parametrize("lb", [3, 4, 5])
def test_ring14_vs_parameter_shift(sv, lb):
    circ = C.WORKLOADS["ring14"]()
    terms = C.z_sum_terms(14)
    st = sv.State(14).reset().run(circ)
    loss, g, drift = st.adjoint_grad(circ, terms, block_qubits=lb)
    _close(g[0], oracle.grad_param_shift(circ, terms))
    assert abs(loss[0] - oracle.loss(circ, terms)) < 1e-4
    assert drift[0] < 1e-4
    assert abs(st.to_numpy()[0][0] - 1) < 1e-4


@pytest.mark.parametrize("lb", [3, 4, 5])
@pytest.mark.parametrize("n,seed", [(6, 1), (9, 2), (12, 3)])
def test_every_kind_vs_oracle_adjoint(sv, lb, n, seed):
    """Random circuits of every kind (controls, two-target kinds, U3 with
    three parameters, phase gates): the oracle's FP64 adjoint (itself pinned
    against parameter shift and central differences) is the reference.
    Observables with X and Y strings exercise the complex co-state."""
    circ = C.random_circuit(n, 90, 40 + seed + lb, max_controls=2 if lb > 3 else 1)
    rng = np.random.default_rng(seed)
    terms = [(float(rng.normal()), int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n))) for _ in range(4)]
    st = sv.State(n).reset().run(circ)
    loss, g, drift = st.adjoint_grad(circ, terms, block_qubits=lb)
    ref_loss, ref, _ = oracle.grad_adjoint(circ, terms)
    _close(g[0], ref)
    assert abs(loss[0] - ref_loss) < 1e-4
    assert drift[0] < 1e-4


def test_blocked_matches_per_gate(sv):
    """Same circuit, same state: the blocked and the per-gate GPU backward
    give the same gradient (to FP32 rounding of the recomputed states)."""
    circ = C.rxry_ring(16, 4, 9)
    terms = C.z_sum_terms(16)
    st = sv.State(16)
    st.reset().run(circ)
    _, g_gate, _ = st.adjoint_grad(circ, terms)
    for lb in (3, 4, 5):
        st.reset().run(circ)
        _, g_blk, d = st.adjoint_grad(circ, terms, block_qubits=lb)
        _close(g_blk[0], g_gate[0], rel=2e-5)
        assert d[0] < 1e-4


def test_batched_rows_weighted(sv):
    """The profiling ladder with per-row inputs and per-row observable
    weights: rows whose parameters differ get their own launches."""
    n, B = 10, 4
    circ, rows = C.profiling_ladder(n, 3, B, seed=12)
    coeff = np.random.default_rng(13).normal(size=(B, n))
    terms = [(1.0, 0, 1 << i) for i in range(n)]
    st = sv.State(n, B)
    st.reset().run(circ, params=rows)
    loss, g, drift = st.adjoint_grad(circ, terms, params=rows, coeff_rows=coeff, block_qubits=5)
    for r in range(B):
        wt = [(float(coeff[r, i]), 0, 1 << i) for i in range(n)]
        ref_loss, ref, _ = oracle.grad_adjoint(circ, wt, params=rows[r])
        _close(g[r], ref)
        assert abs(loss[r] - ref_loss) < 1e-4
    assert np.all(drift < 1e-4)


def test_many_parameters_in_one_block(sv):
    """More derivative slots than one launch holds (64): 150 rotations on
    qubits 0..3 (one 4-qubit block) are split into several launches."""
    b = C._Builder(8)
    rng = np.random.default_rng(5)
    for i in range(150):
        b.gate(["rx", "ry", "rz"][i % 3], [i % 4], values=[rng.uniform(0, 2 * np.pi)])
    for q in range(3):
        b.gate("x", [q + 1], [q])
    circ = b.build("dense_rotations")
    terms = C.z_sum_terms(8)
    st = sv.State(8).reset().run(circ)
    _, g, _ = st.adjoint_grad(circ, terms, block_qubits=4)
    _close(g[0], oracle.grad_param_shift(circ, terms))


def test_bad_block_width(sv):
    circ = C.WORKLOADS["ring14"]()
    st = sv.State(14).reset().run(circ)
    with pytest.raises(svmod.SvError):
        st.adjoint_grad(circ, C.z_sum_terms(14), block_qubits=2)
    st3 = sv.State(3).reset()
    with pytest.raises(svmod.SvError):
        st3.adjoint_grad(C.ghz(3), C.z_sum_terms(3), block_qubits=4)
    with pytest.raises(svmod.SvError):
        st.adjoint_grad(circ, C.z_sum_terms(14), block_qubits=6)
    # a gate wider than the block (two targets, two controls) is refused
    b = C._Builder(6)
    b.gate("rxx", [0, 1], [2, 3], values=[0.3])
    wide = b.build("wide_gate")
    st6 = sv.State(6).reset().run(wide)
    with pytest.raises(svmod.SvError) as e:
        st6.adjoint_grad(wide, C.z_sum_terms(6), block_qubits=3)
    assert e.value.status == 4
