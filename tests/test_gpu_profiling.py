"""The paper's profiling workload on one GPU (Sec. 5, Fig. 3; the appendix
example): an RY input encoding, 3 x [CNOT ring, RY], batch 16, exact <Z_i> of
every qubit, loss sum |<Z_i>|, Adam on the inputs (not the angles).

Parity against the oracle:
* the weighted adjoint (each row its own observable sum_i c[r, i] Z_i) vs the
  oracle's parameter-shift gradient of the same weighted observable, per row
  (relative 1e-4), with rows that share the ansatz angles (one launch for all
  rows) and rows that differ everywhere (one launch per row);
* ExpvalZ forward vs the oracle's <Z_i>, backward vs central differences of
  the oracle;
* five Adam steps on the inputs at 12 qubits vs the same loop on the CPU
  with the oracle's <Z_i> and parameter-shift gradients (loss trajectory and
  final inputs);
* at the paper's sizes (18 and 24 qubits, batch 16): the gradient of sampled
  inputs vs the oracle (18 qubits) and directional derivatives of the loss
  (24 qubits, a property at any size).
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd.autograd import ExpvalZ, MeasureAllZ

pytestmark = pytest.mark.gpu


def _zterms(n, c=None):
    return [(1.0 if c is None else float(c[i]), 0, 1 << i) for i in range(n)]


def _oracle_weighted_grad(circ, row, c):
    return oracle.grad_param_shift(circ, _zterms(circ.n, c), params=row)


@pytest.mark.parametrize("shared", [True, False])
def test_weighted_adjoint_vs_parameter_shift(sv, shared):
    n, B = 9, 4
    circ, rows = C.profiling_ladder(n, 3, B, seed=2)
    rng = np.random.default_rng(3)
    if not shared:
        rows = rows + rng.uniform(-0.3, 0.3, size=rows.shape)
    coeff = rng.normal(size=(B, n))
    st = sv.State(n, B)
    st.reset().run(circ, params=rows)
    loss, grad, drift = st.adjoint_grad(circ, _zterms(n), params=rows, coeff_rows=coeff)
    for r in range(B):
        want = _oracle_weighted_grad(circ, rows[r], coeff[r])
        err = np.linalg.norm(grad[r] - want) / np.linalg.norm(want)
        assert err < 1e-4, (r, err)
        psi = oracle.run(circ, params=rows[r])
        assert abs(loss[r] - oracle.expval_terms(psi, n, _zterms(n, coeff[r]))) < 1e-5
    assert np.all(drift < 1e-4)


@pytest.mark.parametrize("block_qubits,n,fuse", [(None, 8, False), (0, 8, False), (3, 8, False), (5, 8, False),
                                                 (None, 14, True)])
def test_expvalz_forward_and_backward(sv, block_qubits, n, fuse):
    """None: the default (blocked, 4 qubits); 0: the per-gate backward;
    fuse: the fused forward (row-shared gates as matrix-core blocks)."""
    B = 3
    circ, rows = C.profiling_ladder(n, 3, B, seed=4)
    layer = MeasureAllZ(circ, B, block_qubits=block_qubits, fuse=fuse)
    x = torch.tensor(rows, dtype=torch.float64, requires_grad=True)
    z = layer(x)
    for r in range(B):
        want, _ = oracle.expval_z_all(oracle.run(circ, params=rows[r]), n)
        np.testing.assert_allclose(z[r].detach().numpy(), want[:n], atol=2e-6)
    w = torch.tensor(np.random.default_rng(5).normal(size=(B, n)))
    (z * w).sum().backward()
    g = x.grad.numpy()
    h = 1e-4
    for r in range(B):
        for j in (0, 3, n + 2, 2 * n + 5):
            pp, pm = rows[r].copy(), rows[r].copy()
            pp[j] += h
            pm[j] -= h
            fp = oracle.expval_terms(oracle.run(circ, params=pp), n, _zterms(n, w[r].numpy()))
            fm = oracle.expval_terms(oracle.run(circ, params=pm), n, _zterms(n, w[r].numpy()))
            assert abs(g[r, j] - (fp - fm) / (2 * h)) < 1e-4 * max(1.0, abs(g[r, j]))


@pytest.mark.parametrize("shared", [True, False], ids=["shared_ansatz", "all_per_row"])
def test_run_fused_forward(sv, shared):
    """The fused forward of the autograd layers: gates whose angles are equal
    on every row as 5-qubit matrix-core blocks, per-row gates (the input
    encoding) as matrix-core blocks with one matrix per row, in circuit
    order. Equal to the per-gate forward (2e-6) and to the oracle (1e-5) row
    by row."""
    n, B = 14, 3
    circ, rows = C.profiling_ladder(n, 3, B, seed=11)
    if not shared:
        rows = rows + np.random.default_rng(12).uniform(-0.2, 0.2, size=rows.shape)
    a = sv.State(n, B).reset().run(circ, params=rows).to_numpy()
    b = sv.State(n, B).reset().run_fused(circ, params=rows).to_numpy()
    assert np.max(np.abs(a - b)) < 2e-6
    for r in range(B):
        assert np.max(np.abs(b[r] - oracle.run(circ, params=rows[r]))) < 1e-5


def test_run_fused_general_circuit(sv):
    """run_fused on a circuit with two-qubit and controlled gates and shared
    parameters (one fused sweep per block) vs the oracle."""
    circ = C.random_circuit(13, 160, 21)
    b = sv.State(13).reset().run_fused(circ).to_numpy()[0]
    assert np.max(np.abs(b - oracle.run(circ))) < 1e-5


def _cpu_adam_loop(circ, rows, steps, lr):
    """Reference: the same Adam loop with the oracle's <Z_i> and
    parameter-shift gradients, torch's Adam on the CPU."""
    n = circ.n
    B = rows.shape[0]
    x = torch.tensor(rows[:, :n].copy(), requires_grad=True)
    opt = torch.optim.Adam([x], lr=lr)
    theta = rows[:, n:]
    losses = []
    for _ in range(steps):
        opt.zero_grad()
        g = np.zeros((B, n))
        total = 0.0
        for r in range(B):
            p = np.concatenate([x.detach().numpy()[r], theta[r]])
            z, _ = oracle.expval_z_all(oracle.run(circ, params=p), n)
            z = z[:n]
            total += np.abs(z).sum()
            g[r] = oracle.grad_param_shift(circ, _zterms(n, np.sign(z)), params=p)[:n]
        losses.append(total)
        x.grad = torch.tensor(g)
        opt.step()
    return np.array(losses), x.detach().numpy()


def _gpu_adam_loop(sv, circ, rows, steps, lr):
    n = circ.n
    B = rows.shape[0]
    layer = MeasureAllZ(circ, B)
    x = torch.tensor(rows[:, :n].copy(), dtype=torch.float64, requires_grad=True)
    theta = torch.tensor(rows[:, n:])
    opt = torch.optim.Adam([x], lr=lr)
    losses = []
    for _ in range(steps):
        opt.zero_grad()
        z = layer(torch.cat([x, theta], dim=1))
        loss = z.abs().sum()
        losses.append(loss.item())
        loss.backward()
        opt.step()
    return np.array(losses), x.detach().numpy()


def test_adam_on_inputs_matches_cpu_loop(sv):
    circ, rows = C.profiling_ladder(12, 3, 16, seed=6)
    lg, xg = _gpu_adam_loop(sv, circ, rows, 5, lr=0.05)
    lc, xc = _cpu_adam_loop(circ, rows, 5, lr=0.05)
    np.testing.assert_allclose(lg, lc, rtol=1e-5)
    np.testing.assert_allclose(xg, xc, atol=1e-5)
    assert lg[-1] < lg[0]


def test_paper_sizes(sv):
    """18 qubits: the gradient of the paper's loss sum |<Z_i>| at sampled
    rows vs the oracle's parameter shift of sum sign(<Z_i>) Z_i. 24 qubits:
    directional derivatives of a smooth loss sum w <Z> (central differences
    of the GPU forward, h = 5e-3: truncation ~1e-5, complex64 rounding of the
    loss ~1e-4 / 2h; |<Z>| has kinks where <Z_i> crosses 0, which a finite
    difference of that size can straddle) against the adjoint gradient,
    relative 1e-2."""
    for n in (18, 24):
        circ, rows = C.profiling_ladder(n, 3, 16, seed=7)
        layer = MeasureAllZ(circ, 16)
        x = torch.tensor(rows, dtype=torch.float64, requires_grad=True)
        z = layer(x)
        if n == 18:
            z.abs().sum().backward()
            g = x.grad.numpy()
            zc = z.detach().numpy()
            for r in (0, 9):
                want = oracle.grad_param_shift(circ, _zterms(n, np.sign(zc[r])), params=rows[r])
                assert np.max(np.abs(g[r, :n] - want[:n])) < 1e-4 * max(1.0, np.max(np.abs(want[:n])))
        else:
            w = torch.tensor(np.random.default_rng(9).normal(size=(16, n)))
            (z * w).sum().backward()
            g = x.grad.numpy()
            rng = np.random.default_rng(8)
            for _ in range(2):
                d = np.zeros_like(rows)
                d[:, :n] = rng.normal(size=(16, n))
                h = 5e-3
                with torch.no_grad():
                    fp = (layer(torch.tensor(rows + h * d)) * w).sum().item()
                    fm = (layer(torch.tensor(rows - h * d)) * w).sum().item()
                fd = (fp - fm) / (2 * h)
                assert abs(fd - np.sum(g * d)) < 1e-2 * max(1.0, abs(fd))
        layer.state.free()
