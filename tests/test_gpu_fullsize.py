"""Parity at the workloads' own sizes against values the oracle computed
(complex128) and stored under tests/golden by oracle/make_goldens.py, or
against the oracle run here where it finishes in seconds.

* brickwork30 (30 qubits, 890 gates; the launch bench.py times) as plain
  sweeps and fused into 5- and 6-qubit blocks (FP32 and BF16x3 matrix
  cores): every <Z_i>, <sum Z_i> and 1026 sampled amplitudes against the
  oracle's values;
* brickwork24 as plain per-gate sweeps: the full state against the oracle's;
* brickwork32 (32 GiB): every fused mode against the plain sweeps (<Z_i> and
  sampled amplitudes; the oracle cannot hold this state);
* the paper's profiling ladder at 24 qubits, batch 16: every row's gradient
  of sum_i c[r, i] <Z_i> (inputs and angles) against the oracle's.

Bounds come from tests/errmodel.py: B bounds ||dpsi||_2 from the sweeps a
path runs; <Z_i> within 2 B + B^2; ||dpsi|| estimated from the sampled
amplitudes must lie within B. Gradients within 1e-4 relative.
"""

import json
import os

import numpy as np
import pytest
import torch

from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod
from tests import errmodel

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def _free_gib():
    free, _ = torch.cuda.mem_get_info()
    return free / 2 ** 30


def _sampled(st, idx):
    t = st.tensor[0]
    return t[torch.as_tensor(np.asarray(idx, dtype=np.int64), device=t.device)].cpu().numpy().astype(np.complex128)


def _fused_eps(blocks, mode):
    eps = []
    for targets, _ in blocks:
        k = len(targets)
        if mode == svmod.FUSED_BF16X3:
            eps.append(errmodel.eps_bf16x3_block(k))
        else:
            eps.append(errmodel.eps_fp32_block(k))
    return eps


FUSED_CASES = [(5, svmod.FUSED_FP32_MFMA), (5, svmod.FUSED_BF16X3), (6, svmod.FUSED_BF16X3)]


def _check_vs_golden(label, st, g, B):
    n = g["n"]
    z = st.expval_z_all()[0]
    want = np.array(g["expval_z"])
    zb = errmodel.z_bound(B)
    dz = float(np.max(np.abs(z[:n] - want)))
    dsum = abs(float(np.sum(z[:n])) - g["sum_z"])
    amps = _sampled(st, g["amp_index"])
    ref = np.array(g["amp_re"]) + 1j * np.array(g["amp_im"])
    est = errmodel.sampled_norm_estimate(amps - ref, n)
    print(f"{label}: max|d<Z_i>| {dz:.2e} (bound {zb:.2e}), |d<sum Z>| {dsum:.2e} (bound {n * zb:.2e}), "
          f"||dpsi|| from samples {est:.2e} (bound {B:.2e}), max|dpsi_b| {np.max(np.abs(amps - ref)):.2e}")
    assert dz <= zb
    assert dsum <= n * zb
    assert abs(z[n] - g["norm2"]) <= 2 * B + B * B
    assert est <= B


def test_brickwork30_plain_vs_oracle(sv):
    """The benchmark step itself (plain sweeps, then <Z_i>)."""
    g = _golden("brickwork30")
    circ = C.WORKLOADS["brickwork30"]()
    assert len(circ.ops) == g["n_gates"]
    st = svmod.State(30).reset().run(circ)
    B = errmodel.state_bound(errmodel.plain_circuit_eps(circ))
    _check_vs_golden("brickwork30 plain", st, g, B)
    st.free()


@pytest.mark.parametrize("k,mode", FUSED_CASES, ids=["fp32_k5", "bf16x3_k5", "bf16x3_k6"])
def test_brickwork30_fused_vs_oracle(sv, k, mode):
    g = _golden("brickwork30")
    circ = C.WORKLOADS["brickwork30"]()
    blocks = svmod.fuse_plan(circ, k)
    st = svmod.State(30).reset().apply_fused(blocks, mode)
    B = errmodel.state_bound(_fused_eps(blocks, mode))
    _check_vs_golden(f"brickwork30 fused k={k} mode={mode} ({len(blocks)} blocks)", st, g, B)
    st.free()


def test_brickwork24_plain_full_state(sv):
    """The 24-qubit instance of the plain workload gate by gate: the whole
    state against the oracle's (max amplitude error <= 1e-5, ||dpsi||_2 and
    1 - F within the bound)."""
    import oracle

    circ = C.WORKLOADS["brickwork24"]()
    st = svmod.State(24).reset().run(circ)
    out = st.to_numpy()[0].astype(np.complex128)
    ref = oracle.run(circ)
    d = out - ref
    B = errmodel.state_bound(errmodel.plain_circuit_eps(circ))
    err = float(np.max(np.abs(d)))
    dn = float(np.linalg.norm(d))
    infid = 1.0 - abs(np.vdot(ref, out)) ** 2 / np.vdot(out, out).real
    z = st.expval_z_all()[0]
    zr, _ = oracle.expval_z_all(ref, 24)
    print(f"brickwork24 plain: max|dpsi| {err:.2e}, ||dpsi|| {dn:.2e} (bound {B:.2e}), 1-F {infid:.2e} "
          f"(bound {errmodel.infidelity_bound(B):.2e}), max|d<Z>| {np.max(np.abs(z[:24] - zr)):.2e}")
    assert err <= 1e-5
    assert dn <= B
    assert infid <= errmodel.infidelity_bound(B)
    assert np.max(np.abs(z[:24] - zr)) <= 2 * dn + dn * dn
    st.free()


def test_brickwork32_fused_vs_plain(sv):
    """32 qubits (32 GiB): <Z_i> and 1026 seeded amplitudes of every fused
    mode against the plain sweeps, within the sum of both paths' bounds."""
    if _free_gib() < 40:
        pytest.skip("needs 40 GiB of free device memory")
    n = 32
    circ = C.WORKLOADS["fused32"]()
    rng = np.random.Generator(np.random.PCG64(32))
    idx = np.unique(np.concatenate([[0, (1 << n) - 1], rng.integers(0, 1 << n, size=1024)]))
    st = svmod.State(n).reset().run(circ)
    z_plain = st.expval_z_all()[0]
    a_plain = _sampled(st, idx)
    Bp = errmodel.state_bound(errmodel.plain_circuit_eps(circ))
    for k, mode in FUSED_CASES:
        blocks = svmod.fuse_plan(circ, k)
        st.reset().apply_fused(blocks, mode)
        z = st.expval_z_all()[0]
        a = _sampled(st, idx)
        B = Bp + errmodel.state_bound(_fused_eps(blocks, mode))
        dz = float(np.max(np.abs(z[:n] - z_plain[:n])))
        est = errmodel.sampled_norm_estimate(a - a_plain, n)
        print(f"brickwork32 k={k} mode={mode}: max|d<Z_i>| vs plain {dz:.2e} (bound {errmodel.z_bound(B):.2e}), "
              f"||dpsi|| from samples {est:.2e} (bound {B:.2e})")
        assert dz <= errmodel.z_bound(B)
        assert est <= B
    st.free()


@pytest.mark.parametrize("block", [0, svmod.ADJOINT_MFMA], ids=["per_gate", "mfma"])
def test_profiling24_rows_vs_oracle_adjoint(sv, block):
    """The paper's profiling ladder at 24 qubits, batch 16 (per-row inputs,
    shared angles): per row the loss sum_i c[r, i] <Z_i> and its gradient in
    all 96 parameters against the oracle's adjoint, relative 1e-4."""
    g = _golden("profiling24")
    n, B = g["n"], g["batch"]
    circ, rows = C.profiling_ladder(n, 3, B, seed=7)
    coeff = np.array(g["coeff"])
    terms = [(1.0, 0, 1 << i) for i in range(n)]
    st = svmod.State(n, B).reset().run(circ, rows)
    loss, grad, drift = st.adjoint_grad(circ, terms, params=rows, coeff_rows=coeff, block_qubits=block)
    want = np.array(g["grad"])
    worst = 0.0
    for r in range(B):
        rel = float(np.max(np.abs(grad[r] - want[r])) / np.max(np.abs(want[r])))
        worst = max(worst, rel)
        assert rel <= 1e-4, (r, rel)
        assert abs(loss[r] - g["loss"][r]) <= 1e-4 * max(1.0, abs(g["loss"][r]))
    print(f"profiling24 {block}: worst row max|dg|/max|g| {worst:.2e}, max drift {np.max(drift):.2e}")
    st.free()
