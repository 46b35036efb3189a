"""GPU parity of the fused-block sweeps (FP32 MFMA, split BF16x3 MFMA, FP32
vector) against the oracle's unfused gate-by-gate result.

Tolerance: max |psi - psi_ref| <= 1e-5 per amplitude for every mode, and
on the planned circuits ||dpsi||_2 and 1 - F within the rounding-error
bound of the blocks run (tests/errmodel.py: FP32 products round at 2^-24
relative; BF16x3 drops only the lo*lo product and the residuals of the
two-term splits, about 2^-16 relative per product).
"""

import numpy as np
import pytest

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod
from tests import errmodel, pins

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-5
MODES = [svmod.FUSED_FP32_MFMA, svmod.FUSED_BF16X3, svmod.FUSED_VALU]


def _block_bound(blocks, mode):
    eps = []
    for targets, _ in blocks:
        k = len(targets)
        eps.append(errmodel.eps_bf16x3_block(k) if mode == svmod.FUSED_BF16X3 else errmodel.eps_fp32_block(k))
    return errmodel.state_bound(eps)


def _assert_state(out, ref, B, label=""):
    out = out.astype(np.complex128)
    d = out - ref
    dn = float(np.linalg.norm(d))
    infid = 1.0 - abs(np.vdot(ref, out)) ** 2 / np.vdot(out, out).real
    print(f"{label} max|dpsi| {np.max(np.abs(d)):.2e} ||dpsi|| {dn:.2e} (bound {B:.2e}) 1-F {infid:.2e} "
          f"(bound {errmodel.infidelity_bound(B):.2e})")
    assert np.max(np.abs(d)) <= AMP_TOL
    assert dn <= B
    assert infid <= errmodel.infidelity_bound(B)
    return dn


def _upload(sv, n, psi, batch=1):
    st = sv.State(n, batch)
    st.from_numpy(np.tile(psi.astype(np.complex64), (batch, 1)))
    return st


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,targets", [
    (10, (9, 8, 7, 6, 5)),        # targets high: columns = bits 0..4
    (10, (0, 1, 2, 3, 4)),        # targets low: columns = bits 5..9
    (12, (3, 0, 11, 6, 1)),       # scattered, unsorted
    (15, (14, 2, 7, 9, 5)),
    (16, (4, 12, 0, 15, 8)),
    (13, (12, 5, 9, 6, 11)),      # all targets >= 5: direct operand form
    (20, (19, 7, 13, 5, 16)),
    (12, (11, 10, 9, 8, 7)),      # all targets >= 6: wide direct form
    (17, (13, 6, 16, 7, 10)),
])
def test_single_block_random_unitary(sv, mode, n, targets):
    """A Haar-random 32x32 unitary on five ordered targets: pins the MFMA
    operand and result layouts and the tile bit mapping."""
    rng = np.random.default_rng(n * 7 + sum(targets))
    psi0 = pins.random_state(n, rng)
    m = pins.haar_unitary(32, rng)
    st = _upload(sv, n, psi0, batch=2)
    st.apply_fused([(targets, m)], mode)
    ref = psi0.astype(np.complex64).astype(np.complex128)
    oracle.apply_matrix(ref, n, m, list(targets))
    out = st.to_numpy()
    for r in range(2):
        assert np.max(np.abs(out[r] - ref)) <= AMP_TOL


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_small_blocks_padded(sv, mode, k):
    n = 11
    rng = np.random.default_rng(50 + k)
    psi0 = pins.random_state(n, rng)
    targets = tuple(int(x) for x in rng.permutation(n)[:k])
    m = pins.haar_unitary(1 << k, rng)
    st = _upload(sv, n, psi0)
    st.apply_fused([(targets, m)], mode)
    ref = psi0.astype(np.complex64).astype(np.complex128)
    oracle.apply_matrix(ref, n, m, list(targets))
    assert np.max(np.abs(st.to_numpy()[0] - ref)) <= AMP_TOL


@pytest.mark.parametrize("mode", MODES[:2])
@pytest.mark.parametrize("n,targets", [
    (10, (9, 8, 7, 6, 5)),        # wide form
    (12, (5, 11, 7, 9, 6)),       # direct form
    (13, (3, 0, 12, 6, 1)),       # LDS-staged form
    (11, (4, 9)),                 # padded to five qubits
])
def test_per_row_matrices(sv, mode, n, targets):
    """sv_apply_fused_rows: every row of a batch of 3 (different states) with
    its own Haar-random matrix, each row against the oracle; two blocks in a
    row, the second on other targets."""
    B = 3
    rng = np.random.default_rng(n * 11 + len(targets))
    psi0 = [pins.random_state(n, rng) for _ in range(B)]
    k = len(targets)
    ms = np.stack([pins.haar_unitary(1 << k, rng) for _ in range(B)])
    t2 = tuple(int(x) for x in rng.permutation(n)[:5])
    ms2 = np.stack([pins.haar_unitary(32, rng) for _ in range(B)])
    st = sv.State(n, B)
    st.from_numpy(np.stack(psi0).astype(np.complex64))
    st.apply_fused_rows([(targets, ms), (t2, ms2)], mode)
    out = st.to_numpy()
    for r in range(B):
        ref = psi0[r].astype(np.complex64).astype(np.complex128)
        oracle.apply_matrix(ref, n, ms[r], list(targets))
        oracle.apply_matrix(ref, n, ms2[r], list(t2))
        assert np.max(np.abs(out[r] - ref)) <= AMP_TOL


def test_per_row_matrices_refusals(sv):
    n, B = 12, 2
    st = sv.State(n, B).reset()
    rng = np.random.default_rng(5)
    m5 = np.stack([pins.haar_unitary(32, rng) for _ in range(B)])
    with pytest.raises(svmod.SvError) as e:
        st.apply_fused_rows([((0, 1, 2, 3, 4), m5)], svmod.FUSED_VALU)
    assert e.value.status == 4
    m6 = np.stack([pins.haar_unitary(64, rng) for _ in range(B)])
    with pytest.raises(svmod.SvError) as e:
        st.apply_fused_rows([((11, 10, 9, 8, 7, 6), m6)], svmod.FUSED_BF16X3)
    assert e.value.status == 4
    with pytest.raises(ValueError):
        st.apply_fused_rows([((0, 1, 2, 3, 4), m5[:1])], svmod.FUSED_FP32_MFMA)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", [10, 14, 18])
def test_planned_brickwork_vs_unfused_oracle(sv, mode, n):
    """The brickwork circuit fused into <= 5-qubit blocks by the planner and
    run block by block equals the oracle's gate-by-gate state."""
    circ = C.brickwork_u3_cz(n, 20, 3)
    blocks = svmod.fuse_plan(circ, 5)
    assert len(blocks) < len(circ.ops) / 4
    st = sv.State(n).reset()
    st.apply_fused(blocks, mode)
    ref = oracle.run(circ)
    _assert_state(st.to_numpy()[0], ref, _block_bound(blocks, mode), f"n={n} mode={mode}")


def test_mfma_needs_ten_qubits_valu_does_not(sv):
    n = 8
    rng = np.random.default_rng(3)
    m = pins.haar_unitary(32, rng)
    st = sv.State(n).reset()
    with pytest.raises(svmod.SvError) as e:
        st.apply_fused([((0, 1, 2, 3, 4), m)], svmod.FUSED_FP32_MFMA)
    assert e.value.status == 1
    st.apply_fused([((0, 1, 2, 3, 4), m)], svmod.FUSED_VALU)
    ref = oracle.basis_state(n, 0)
    oracle.apply_matrix(ref, n, m, [0, 1, 2, 3, 4])
    assert np.max(np.abs(st.to_numpy()[0] - ref)) <= AMP_TOL


@pytest.fixture(scope="module")
def fused24_reference():
    circ = C.WORKLOADS["fused24"]()
    return circ, oracle.run(circ)


@pytest.mark.parametrize("mode", MODES)
def test_fused24_error_vs_fp64_oracle(sv, fused24_reference, mode):
    """24-qubit instance of the fusion workload: FP32 MFMA and BF16x3 against
    the complex128 oracle (max amplitude error, ||dpsi||_2, infidelity,
    <sum Z> error), next to the plain per-gate path."""
    circ, ref = fused24_reference
    n = circ.n
    blocks = svmod.fuse_plan(circ, 5)
    st = sv.State(n).reset()
    st.apply_fused(blocks, mode)
    out = st.to_numpy()[0]
    dn = _assert_state(out, ref, _block_bound(blocks, mode), f"fused24 mode {mode}:")
    z = st.expval_z_all()[0]
    zr, _ = oracle.expval_z_all(ref, n)
    print(f"mode {mode}: d<sumZ> {abs(z[:n].sum() - zr.sum()):.2e}")
    assert abs(z[:n].sum() - zr.sum()) <= n * (2 * dn + dn * dn) + 1e-12


@pytest.mark.parametrize("n,targets", [
    (12, (11, 10, 9, 8, 7, 6)),       # the smallest state: one tile row per wave
    (12, (6, 7, 8, 9, 10, 11)),       # reversed target order
    (18, (17, 6, 12, 9, 15, 7)),      # scattered, unsorted
    (21, (20, 19, 6, 13, 8, 16)),
])
def test_six_qubit_block_random_unitary(sv, n, targets):
    """A Haar-random 64x64 unitary on six targets >= 6 (BF16x3 six-qubit
    form): pins the 128x128 operand layout, both output halves and the
    even/odd column accumulators, on two batch rows."""
    rng = np.random.default_rng(n * 11 + sum(targets))
    psi0 = pins.random_state(n, rng)
    m = pins.haar_unitary(64, rng)
    st = _upload(sv, n, psi0, batch=2)
    st.apply_fused([(targets, m)], svmod.FUSED_BF16X3)
    ref = psi0.astype(np.complex64).astype(np.complex128)
    oracle.apply_matrix(ref, n, m, list(targets))
    out = st.to_numpy()
    for r in range(2):
        assert np.max(np.abs(out[r] - ref)) <= AMP_TOL


@pytest.mark.parametrize("n", [12, 16, 20])
def test_planned_six_qubit_brickwork_vs_unfused_oracle(sv, n):
    """Brickwork planned with max_k = 6 (six-qubit blocks off qubits 0..5,
    five-qubit blocks elsewhere) in BF16x3 equals the oracle's state, with
    fewer blocks than the five-qubit plan."""
    circ = C.brickwork_u3_cz(n, 20, 3)
    blocks = svmod.fuse_plan(circ, 6)
    assert any(len(t) == 6 for t, _ in blocks)
    assert len(blocks) < len(svmod.fuse_plan(circ, 5))
    st = sv.State(n).reset()
    st.apply_fused(blocks, svmod.FUSED_BF16X3)
    ref = oracle.run(circ)
    _assert_state(st.to_numpy()[0], ref, _block_bound(blocks, svmod.FUSED_BF16X3), f"k6 n={n}")


def test_six_qubit_block_conditions(sv):
    rng = np.random.default_rng(4)
    m = pins.haar_unitary(64, rng)
    st = sv.State(14).reset()
    for mode in (svmod.FUSED_FP32_MFMA, svmod.FUSED_VALU):
        with pytest.raises(svmod.SvError) as e:
            st.apply_fused([((13, 12, 11, 10, 9, 8), m)], mode)
        assert e.value.status == 4                     # unsupported
    with pytest.raises(svmod.SvError) as e:
        st.apply_fused([((13, 12, 11, 10, 9, 5), m)], svmod.FUSED_BF16X3)
    assert e.value.status == 4
    with pytest.raises(svmod.SvError) as e:
        sv.State(11).reset().apply_fused([((10, 9, 8, 7, 6, 5), m)], svmod.FUSED_BF16X3)
    assert e.value.status in (1, 4)
