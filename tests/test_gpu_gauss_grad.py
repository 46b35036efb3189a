"""GPU parity of the differentiable Gaussian shot estimate (Sec. 4.3.2 with
the normals held fixed; the backward is the adjoint of Sec. 4.4 started from
a diagonal observable).

* sv_gaussian_expval_z vs the oracle's estimate on the same amplitudes (the
  GPU state read back and widened to complex128, so only the FP64 summation
  order differs): 1e-10.
* sv_gaussian_expval_z_backward vs the oracle's weights w_b = dF/d|psi_b|^2
  on the same amplitudes, element by element (relative 1e-9), including
  amplitudes that are exactly 0 (the 1/sqrt(p) term is taken as 0 there on
  both sides).
* sv_adjoint_grad_diag: per-gate and blocked agree; for W = diag(sign
  patterns of Z_i) it equals the Pauli adjoint of sum_i Z_i.
* End to end (GaussianExpvalZ): the gradient of F = sum_i c_i E_i with
  respect to inputs and angles vs central differences of the oracle's
  pipeline (oracle state, oracle estimate, the same normals), relative 1e-4;
  at 22 qubits, directional derivatives of the GPU forward (a property at any
  size).
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd.autograd import GaussianExpvalZ

pytestmark = pytest.mark.gpu


def _state(sv, n, seed, zeros=()):
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi[list(zeros)] = 0.0
    psi /= np.linalg.norm(psi)
    st = sv.State(n).from_numpy(psi.astype(np.complex64))
    return st, st.to_numpy()[0].astype(np.complex128)


@pytest.mark.parametrize("n,shots", [(6, 50.0), (11, 1000.0), (14, 1e6)])
def test_estimate_matches_oracle(sv, n, shots):
    st, psi = _state(sv, n, n)
    z = np.random.default_rng(100 + n).normal(size=1 << n)
    est = st.gaussian_expval_z(torch.tensor(z, device="cuda"), shots)
    np.testing.assert_allclose(est, oracle.gaussian_z(psi, n, z, shots), atol=1e-10)


@pytest.mark.parametrize("n,shots,zeros", [(5, 30.0, ()), (10, 500.0, (0, 7, 513)), (13, 1e4, (8191,))])
def test_weights_match_oracle(sv, n, shots, zeros):
    st, psi = _state(sv, n, 2 * n, zeros)
    rng = np.random.default_rng(200 + n)
    z = rng.normal(size=1 << n)
    g = rng.normal(size=n)
    w = st.gaussian_expval_z_backward(torch.tensor(z, device="cuda"), shots, g).cpu().numpy()
    want = oracle.gaussian_z_weights(psi, n, z, shots, g)
    np.testing.assert_allclose(w, want, rtol=1e-9, atol=1e-9 * np.max(np.abs(want)))


def test_diag_adjoint_equals_pauli_adjoint(sv):
    """W = diag(sum_i s_i(b)) is the observable sum_i Z_i: the diagonal
    adjoint (per gate and blocked) equals the Pauli adjoint."""
    n = 9
    circ = C.rxry_ring(n, 2, 4)
    st = sv.State(n)
    st.reset().run(circ)
    b = np.arange(1 << n)
    w = sum(1.0 - 2.0 * ((b >> i) & 1) for i in range(n)).astype(np.float64)
    wt = torch.tensor(w, device="cuda").reshape(1, -1).contiguous()
    loss_p, grad_p, _ = st.adjoint_grad(circ, C.z_sum_terms(n))
    for bq in (0, 4):
        st.reset().run(circ)
        loss_d, grad_d, drift = st.adjoint_grad_diag(circ, wt, block_qubits=bq)
        np.testing.assert_allclose(loss_d, loss_p, atol=1e-6)
        np.testing.assert_allclose(grad_d, grad_p, atol=1e-6)
        assert drift[0] < 1e-5


def _oracle_F(circ, rows, normals, shots, c):
    tot = 0.0
    for r in range(rows.shape[0]):
        psi = oracle.run(circ, params=rows[r])
        tot += float(np.dot(c[r], oracle.gaussian_z(psi, circ.n, normals[r], shots)))
    return tot


@pytest.mark.parametrize("block_qubits", [0, 4])
def test_end_to_end_gradient_vs_oracle_differences(sv, block_qubits):
    n, B, shots = 8, 2, 200.0
    circ, rows = C.profiling_ladder(n, 2, B, seed=13)
    rng = np.random.default_rng(14)
    normals = rng.normal(size=(B, 1 << n))
    c = rng.normal(size=(B, n))
    st = sv.State(n, B)
    x = torch.tensor(rows, dtype=torch.float64, requires_grad=True)
    e = GaussianExpvalZ.apply(x, circ, st, torch.tensor(normals, device="cuda"), shots, block_qubits, False)
    (e * torch.tensor(c)).sum().backward()
    g = x.grad.numpy()
    h = 1e-5
    for r in range(B):
        for j in (0, 3, n + 1, 2 * n - 1):
            rp, rm = rows.copy(), rows.copy()
            rp[r, j] += h
            rm[r, j] -= h
            fd = (_oracle_F(circ, rp, normals, shots, c) - _oracle_F(circ, rm, normals, shots, c)) / (2 * h)
            assert abs(g[r, j] - fd) < 1e-4 * max(1.0, abs(fd)), (r, j, g[r, j], fd)


def test_gradient_at_22_qubits_directional(sv):
    """Directional derivatives of the GPU forward (central differences,
    h = 1e-3) against the adjoint gradient, relative 1e-2."""
    n, B, shots = 22, 2, 1e4
    circ, rows = C.profiling_ladder(n, 2, B, seed=15)
    rng = np.random.default_rng(16)
    normals = torch.tensor(rng.normal(size=(B, 1 << n)), device="cuda")
    c = torch.tensor(rng.normal(size=(B, n)))
    st = sv.State(n, B)
    x = torch.tensor(rows, dtype=torch.float64, requires_grad=True)
    (GaussianExpvalZ.apply(x, circ, st, normals, shots, 4, True) * c).sum().backward()
    g = x.grad.numpy()
    for _ in range(2):
        d = rng.normal(size=rows.shape)
        h = 1e-3
        with torch.no_grad():
            fp = (GaussianExpvalZ.apply(torch.tensor(rows + h * d), circ, st, normals, shots, 4, True) * c).sum().item()
            fm = (GaussianExpvalZ.apply(torch.tensor(rows - h * d), circ, st, normals, shots, 4, True) * c).sum().item()
        fd = (fp - fm) / (2 * h)
        assert abs(fd - np.sum(g * d)) < 1e-2 * max(1.0, abs(fd)), (fd, np.sum(g * d))
    st.free()


def test_gaussian_z_rejects_bad_arguments(sv):
    st = sv.State(6)
    z = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(sv.SvError):
        st.gaussian_expval_z(z, -1.0)
    with pytest.raises(sv.SvError):
        st.gaussian_expval_z(z, 10.0, row=3)
