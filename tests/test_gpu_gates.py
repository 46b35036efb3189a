"""GPU parity of the plain gate sweeps, state reset and Z/Pauli reductions
against the CPU oracle (through the C ABI).

Tolerances: amplitudes are complex64 on the GPU and complex128 in the
oracle. Each gate rounds every amplitude once in FP32 (relative 2^-24 per
operation, a few operations per output), so after G gates the error is
about sqrt(G) * 1e-7 in norm; the stated bound is max |psi - psi_ref| <= 1e-5
per amplitude. Expectation values of an observable O differ by at most
2 ||O|| ||psi - psi_ref||_2."""

import numpy as np
import pytest

import oracle
from paper_2511_19291_amd import circuits as C
from tests import pins

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-5


def _upload(sv, n, psi, batch=1):
    st = sv.State(n, batch)
    st.from_numpy(np.tile(psi.astype(np.complex64), (batch, 1)))
    return st


def _ref_start(psi):
    return psi.astype(np.complex64).astype(np.complex128)


@pytest.mark.parametrize("n,idx,batch", [(1, 0, 1), (1, 1, 3), (5, 17, 2), (12, 4095, 1), (16, 12345, 2)])
def test_reset_basis(sv, n, idx, batch):
    st = sv.State(n, batch).reset(idx)
    out = st.to_numpy()
    ref = np.zeros((batch, 1 << n), dtype=np.complex64)
    ref[:, idx] = 1
    np.testing.assert_array_equal(out, ref)


KINDS_1Q = ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "sx", "rx", "ry", "rz", "p", "u3"]
KINDS_2Q = ["swap", "rxx", "ryy", "rzz"]


@pytest.mark.parametrize("n", [1, 2, 3, 6, 9, 11])
def test_every_kind_every_target(sv, n):
    """Every kind on every target (and every ordered target pair for 2-qubit
    kinds), each with 0 or 1 control: covers the float4, float2, pair-in-lane
    and diagonal kernel forms, including qubit 0 and the top qubit."""
    rng = np.random.default_rng(n)
    psi0 = pins.random_state(n, rng)
    st = _upload(sv, n, psi0)
    ref = _ref_start(psi0)
    ops = []
    b = C._Builder(n)
    for kind in KINDS_1Q:
        for t in range(n):
            for ctrl in ([], [int(rng.integers(0, n))]):
                if ctrl and (ctrl[0] == t or n < 2):
                    continue
                b.gate(kind, [t], ctrl, rng.uniform(0, 2 * np.pi, C.N_PARAMS[kind]))
    if n >= 2:
        for kind in KINDS_2Q:
            for t0 in range(n):
                for t1 in range(n):
                    if t0 == t1:
                        continue
                    b.gate(kind, [t0, t1], [], rng.uniform(0, 2 * np.pi, C.N_PARAMS[kind]))
    circ = b.build("all_kinds")
    st.run(circ)
    oracle.run(circ, psi=ref)
    out = st.to_numpy()[0]
    assert np.max(np.abs(out - ref)) <= AMP_TOL


@pytest.mark.parametrize("n,seed", [(4, 1), (7, 2), (10, 3), (13, 4), (17, 5)])
def test_random_circuits(sv, n, seed):
    """Random kinds, targets and 0..2 controls, from |0..0>."""
    circ = C.random_circuit(n, 200, seed)
    st = sv.State(n).reset().run(circ)
    ref = oracle.run(circ)
    assert np.max(np.abs(st.to_numpy()[0] - ref)) <= AMP_TOL


@pytest.mark.parametrize("n", [7, 12])
def test_low_qubit_access_forms(sv, n):
    """Controls and targets on the lowest qubits select the shuffle, odd-lane,
    pair-in-lane and masked-diagonal forms: CNOT/CZ/controlled U3 from qubit
    0 to every target, targets 1..6 with controls above and below 7, and
    two-qubit gates with a target at qubit 0."""
    rng = np.random.default_rng(40 + n)
    psi0 = pins.random_state(n, rng)
    st = _upload(sv, n, psi0)
    ref = _ref_start(psi0)
    b = C._Builder(n)
    for t in range(1, n):
        b.gate("x", [t], [0])
        b.gate("z", [t], [0])
        b.gate("u3", [t], [0], rng.uniform(0, 2 * np.pi, 3))
        b.gate("p", [t], [0], [rng.uniform(0, 2 * np.pi)])
        b.gate("rz", [t], [0], [rng.uniform(0, 2 * np.pi)])
    for t in range(1, min(7, n)):
        b.gate("u3", [t], [], rng.uniform(0, 2 * np.pi, 3))
        if t != n - 1:
            b.gate("ry", [t], [n - 1], [rng.uniform(0, 2 * np.pi)])
        b.gate("rx", [t], [(t + 1) % n if (t + 1) % n != t else 0], [rng.uniform(0, 2 * np.pi)])
    for t in range(1, n):
        b.gate("rxx", [0, t], [], [rng.uniform(0, 2 * np.pi)])
        b.gate("swap", [t, 0])
        b.gate("rzz", [t, 0], [], [rng.uniform(0, 2 * np.pi)])
    b.gate("x", [0], [n - 1])
    b.gate("z", [0], [1, 2])
    circ = b.build("low_forms")
    st.run(circ)
    oracle.run(circ, psi=ref)
    assert np.max(np.abs(st.to_numpy()[0] - ref)) <= AMP_TOL


def test_three_controls(sv):
    n = 8
    rng = np.random.default_rng(8)
    b = C._Builder(n)
    for q in range(n):
        b.gate("h", [q])
    for _ in range(30):
        w = rng.permutation(n)
        kind = str(rng.choice(["x", "u3", "rzz", "p", "swap"]))
        nt = C.N_TARGETS[kind]
        b.gate(kind, list(w[:nt]), list(w[nt:nt + 3]), rng.uniform(0, 2 * np.pi, C.N_PARAMS[kind]))
    circ = b.build("c3")
    st = sv.State(n).reset().run(circ)
    assert np.max(np.abs(st.to_numpy()[0] - oracle.run(circ))) <= AMP_TOL


def test_hea12_full_state_and_z0(sv):
    """12-qubit hardware-efficient ansatz (4 x [RY, RZ, CNOT ladder]): the
    full 4096-amplitude state and <Z_0>."""
    circ = C.WORKLOADS["hea12"]()
    st = sv.State(12).reset().run(circ)
    ref = oracle.run(circ)
    assert np.max(np.abs(st.to_numpy()[0] - ref)) <= AMP_TOL
    z = st.expval_z_all()[0]
    zr, nrm = oracle.expval_z_all(ref, 12)
    np.testing.assert_allclose(z[:12], zr, atol=2e-5)
    assert abs(z[12] - 1) < 1e-5


@pytest.mark.parametrize("n", [16, 20])
def test_brickwork_full_state(sv, n):
    """The U3 + alternating-CZ brickwork (20 layers) at sizes the oracle
    finishes in seconds; spans many kernel tiles."""
    circ = C.brickwork_u3_cz(n, 20, 2)
    st = sv.State(n).reset().run(circ)
    ref = oracle.run(circ)
    out = st.to_numpy()[0]
    assert np.max(np.abs(out - ref)) <= AMP_TOL
    z = st.expval_z_all()[0]
    zr, _ = oracle.expval_z_all(ref, n)
    dpsi = np.linalg.norm(out - ref)
    assert np.max(np.abs(z[:n] - zr)) <= 2 * dpsi + 1e-12


def test_batch_rows_and_per_row_params(sv):
    """batch > 1 with shared params (every row equal) and with per-row params
    (each row its own circuit instance)."""
    circ = C.encoded_ansatz(9, 3, np.random.default_rng(3))
    B = 5
    rng = np.random.default_rng(4)
    P = np.tile(circ.params, (B, 1))
    P[:, list(circ.feature_idx)] = rng.uniform(-np.pi, np.pi, size=(B, len(circ.feature_idx)))
    st = sv.State(9, B).reset().run(circ, params=P)
    out = st.to_numpy()
    for r in range(B):
        ref = oracle.run(circ, params=P[r])
        assert np.max(np.abs(out[r] - ref)) <= AMP_TOL
    st2 = sv.State(9, B).reset().run(circ)
    out2 = st2.to_numpy()
    ref = oracle.run(circ)
    for r in range(B):
        assert np.max(np.abs(out2[r] - ref)) <= AMP_TOL


def test_apply_gate_matrix_forms(sv):
    """sv_apply_gate with explicit matrices: Haar-random dense 2x2 and 4x4,
    the adjoint flag, per-row matrices, and the unitarity check."""
    n = 10
    rng = np.random.default_rng(12)
    psi0 = pins.random_state(n, rng)
    st = _upload(sv, n, psi0)
    ref = _ref_start(psi0)
    for _ in range(20):
        k = int(rng.integers(1, 3))
        w = [int(x) for x in rng.permutation(n)[: k + 1]]
        m = pins.haar_unitary(1 << k, rng)
        adj = bool(rng.integers(0, 2))
        st.apply_gate(m, w[:k], w[k:], adjoint=adj)
        oracle.apply_matrix(ref, n, m.conj().T.copy() if adj else m, w[:k], w[k:])
    assert np.max(np.abs(st.to_numpy()[0] - ref)) <= AMP_TOL
    bad = np.array([[1, 0], [0, 2]], dtype=np.complex128)
    with pytest.raises(sv.SvError) as e:
        st.apply_gate(bad, [0], check_unitary=True)
    assert e.value.status == 8
    # per-row matrices
    B = 3
    st = sv.State(6, B).reset()
    ms = np.stack([pins.haar_unitary(2, rng) for _ in range(B)])
    st.apply_gate(ms, [4])
    out = st.to_numpy()
    for r in range(B):
        ref = oracle.basis_state(6, 0)
        oracle.apply_matrix(ref, 6, ms[r], [4])
        assert np.max(np.abs(out[r] - ref)) <= AMP_TOL


def test_validation_errors_leave_state(sv):
    st = sv.State(4).reset()
    h = np.eye(2)
    for targets, controls, code in [([4], [], 2), ([-1], [], 2), ([1], [1], 3), ([0, 0], [], 3),
                                    ([0, 1, 2], [], 4), ([0], [1, 2, 3, 0], 4)]:
        m = np.eye(1 << len(targets))
        with pytest.raises(sv.SvError) as e:
            st.apply_gate(m, targets, controls)
        assert e.value.status == code, (targets, controls)
    out = st.to_numpy()[0]
    assert out[0] == 1 and np.count_nonzero(out) == 1
    del h


@pytest.mark.parametrize("n", [1, 3, 8, 9, 12, 15])
def test_z_all_and_pauli_strings(sv, n):
    """<Z_i> for every qubit in one sweep (tile sizes 2^n for n < 9, else up
    to 2^14 with bits above the tile from the block index) and random Pauli
    strings with X/Y/Z parts, against the oracle on the same state."""
    rng = np.random.default_rng(100 + n)
    psi0 = pins.random_state(n, rng)
    B = 2
    st = _upload(sv, n, psi0, batch=B)
    ref = _ref_start(psi0)
    z = st.expval_z_all()
    zr, nrm = oracle.expval_z_all(ref, n)
    for r in range(B):
        np.testing.assert_allclose(z[r, :n], zr, atol=1e-12)
        assert abs(z[r, n] - nrm) < 1e-12
    terms = [(float(rng.normal()), int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n))) for _ in range(19)]
    terms += [(1.0, 0, 0), (0.5, (1 << n) - 1, 0), (-2.0, 0, (1 << n) - 1)]
    out = st.expval(terms)
    for t, (c, x, zm) in enumerate(terms):
        exp = c * oracle.expval_pauli(ref, n, x, zm)[0]
        for r in range(B):
            assert abs(out[r, t] - exp) < 1e-12, (t, x, zm)


def test_reductions_bitwise_deterministic(sv):
    n = 18
    circ = C.brickwork_u3_cz(n, 4, 9)
    st = sv.State(n).reset().run(circ)
    a = st.expval_z_all()
    b = st.expval_z_all()
    terms = [C.pauli_term(1.0, "X0 Y5 Z17"), C.pauli_term(0.3, "Z2 Z3")]
    c = st.expval(terms)
    d = st.expval(terms)
    assert np.array_equal(a, b) and np.array_equal(c, d)


def test_ghz_and_qft_closed_forms(sv):
    n = 14
    st = sv.State(n).reset().run(C.ghz(n))
    out = st.to_numpy()[0]
    ref = np.zeros(1 << n)
    ref[0] = ref[-1] = 1 / np.sqrt(2)
    assert np.max(np.abs(out - ref)) < 1e-6
    n, j = 9, 300
    st = sv.State(n).reset().run(C.qft(n, j))
    k = np.arange(1 << n)
    ref = np.exp(2j * np.pi * j * k / (1 << n)) / np.sqrt(1 << n)
    assert np.max(np.abs(st.to_numpy()[0] - ref)) < 1e-5


def test_permutations_exact(sv):
    """CNOT/CZ on basis states are exact (+-1 in a single amplitude) even in
    complex64."""
    n = 12
    rng = np.random.default_rng(77)
    b = C._Builder(n)
    for q in range(n - 1):
        b.gate("x", [q + 1], [q])
    b.gate("x", [0], [n - 1])
    for q in range(0, n - 1, 2):
        b.gate("z", [q + 1], [q])
    circ = b.build("perm")
    for _ in range(4):
        j = int(rng.integers(0, 1 << n))
        st = sv.State(n).reset(j).run(circ)
        ref = oracle.basis_state(n, j)
        oracle.run(circ, psi=ref)
        np.testing.assert_array_equal(st.to_numpy()[0], ref.astype(np.complex64))
