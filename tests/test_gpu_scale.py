"""Full-size and edge cases on the GPU, checked by properties that hold at
any size (the oracle cannot hold these states in seconds):

* the benchmark workload itself (30-qubit brickwork, the launch
  configuration bench.py times): the forward circuit followed by its inverse
  returns |0..0>, the norm stays 1, and sampled amplitudes of a shallow
  prefix match the oracle computed amplitude by amplitude;
* the largest state the library accepts (34 qubits, 128 GiB) and 33 qubits:
  GHZ closed form at sampled amplitudes, <Z_i> = 0, fused blocks at the top
  qubits;
* degenerate inputs: empty circuits, one-qubit states, empty fused lists.
"""

import numpy as np
import pytest

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod

pytestmark = pytest.mark.gpu


def _free_gib():
    import torch
    free, _ = torch.cuda.mem_get_info()
    return free / 2 ** 30


def test_brickwork30_round_trip_and_norm(sv):
    """bench.py's workload: 890 plain sweeps then the 890 inverse gates give
    back e_0 (every kernel form, every target); the norm after the forward
    pass is 1."""
    circ = C.brickwork_u3_cz(30, 20, 2)
    st = sv.State(30).reset().run(circ)
    z = st.expval_z_all()[0]
    assert abs(z[30] - 1) < 1e-4
    st.run(C.inverse(circ))
    import torch
    t = st.tensor[0]
    assert abs(t[0].item() - 1) < 1e-4
    assert float(torch.linalg.vector_norm(t[1:]).item()) < 1e-3


def test_brickwork30_prefix_sampled_amplitudes(sv):
    """The first layer of the 30-qubit workload is a product of U3 gates
    followed by CZs: every amplitude is a closed form the oracle evaluates
    one by one (product of 1-qubit columns times the CZ sign)."""
    full = C.brickwork_u3_cz(30, 20, 2)
    n = 30
    first = [op for op in full.ops[: n + 15]]      # U3 on every qubit, then 15 CZ
    circ = C.Circuit(n, first, full.params)
    st = sv.State(n).reset().run(circ)
    cols = [oracle.gate_matrix("u3", [full.params[i] for i in op.params])[:, 0] for op in first[:n]]
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 1 << n, size=64)
    out = st.tensor[0][torch_index(idx)].cpu().numpy()
    for b, got in zip(idx, out):
        amp = 1.0 + 0j
        for q in range(n):
            amp *= cols[q][(int(b) >> q) & 1]
        for op in first[n:]:
            if (int(b) >> op.targets[0]) & 1 and (int(b) >> op.controls[0]) & 1:
                amp = -amp
        assert abs(got - amp) < 1e-6


def torch_index(idx):
    import torch
    return torch.as_tensor(np.asarray(idx, dtype=np.int64), device="cuda")


@pytest.mark.parametrize("n", [33, 34])
def test_largest_states_ghz(sv, n):
    """GHZ on 33 and 34 qubits (64 / 128 GiB): both non-zero amplitudes are
    1/sqrt 2, sampled others are 0, every <Z_i> = 0, norm 1. Exercises 64-bit
    index arithmetic in every form (targets and controls up to qubit 33)."""
    if _free_gib() < (8 << (n - 30)) + 4:
        pytest.skip("not enough device memory for this state")
    st = sv.State(n).reset().run(C.ghz(n))
    t = st.tensor[0]
    r2 = 1 / np.sqrt(2)
    assert abs(t[0].item() - r2) < 1e-6 and abs(t[(1 << n) - 1].item() - r2) < 1e-6
    rng = np.random.default_rng(n)
    idx = rng.integers(1, (1 << n) - 1, size=32)
    assert np.all(np.abs(t[torch_index(idx)].cpu().numpy()) == 0)
    z = st.expval_z_all()[0]
    assert np.max(np.abs(z[:n])) < 1e-6 and abs(z[n] - 1) < 1e-6
    # a fused 5-qubit block on the top qubits, then its inverse
    rng = np.random.default_rng(1)
    from tests import pins
    m = pins.haar_unitary(32, rng)
    top = (n - 1, n - 2, n - 3, n - 5, n - 8)
    st.apply_fused([(top, m)], svmod.FUSED_FP32_MFMA)
    st.apply_fused([(top, m.conj().T.copy())], svmod.FUSED_FP32_MFMA)
    assert abs(t[0].item() - r2) < 1e-5 and abs(t[(1 << n) - 1].item() - r2) < 1e-5
    st.free()
    del st, t
    import torch
    torch.cuda.empty_cache()


def test_degenerate_inputs(sv):
    st = sv.State(1).reset()
    st.run(C.Circuit(1, [], np.zeros(0)))                 # empty circuit
    assert np.array_equal(st.to_numpy()[0], np.array([1, 0], dtype=np.complex64))
    st.apply_fused([], svmod.FUSED_VALU)                   # empty block list
    h = oracle.gate_matrix("h")
    st.apply_gate(h, [0])
    np.testing.assert_allclose(st.to_numpy()[0], [2 ** -0.5, 2 ** -0.5], atol=1e-7)
    z = st.expval_z_all()[0]
    assert abs(z[0]) < 1e-7 and abs(z[1] - 1) < 1e-7
    x = st.expval([C.pauli_term(1.0, "X0")])
    assert abs(x[0, 0] - 1) < 1e-6
    # gradients of a circuit with no parameters: loss only
    circ = C.ghz(3)
    st3 = sv.State(3).reset().run(circ)
    loss, g, drift = st3.adjoint_grad(circ, C.z_sum_terms(3))
    assert g.shape == (1, 0) and abs(loss[0]) < 1e-6 and drift[0] < 1e-6
