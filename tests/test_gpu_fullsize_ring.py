"""The differentiation workload at its own size (28 qubits, 560 parameters,
random angles and the small-angle variant) against the oracle: the
matrix-core and per-gate adjoint gradients against the oracle's adjoint
gradient of every parameter and its parameter-shift values
(tests/golden/ring28*.json, written by oracle/make_goldens.py), and against
parameter shift run on the GPU for 16 sampled parameters. Gradients within
1e-4 relative; GPU parameter-shift values within the rounding-error bound of
two losses (tests/errmodel.py).
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


def _ring_check(name, sv_block, lam):
    g = _golden(name)
    circ = C.WORKLOADS[name]()
    n = circ.n
    assert circ.n_params == g["n_params"] == 560
    terms = C.z_sum_terms(n)
    st = svmod.State(n).reset().run(circ)
    loss, grad, drift = st.adjoint_grad(circ, terms, lambda_tensor=lam, block_qubits=sv_block)
    want = np.array(g["grad"])
    got = grad[0]
    rel = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    rel_max = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    sp = np.array(g["shift_params"])
    rel_shift = float(np.max(np.abs(got[sp] - np.array(g["shift_grad"]))) / np.max(np.abs(want)))
    print(f"{name} backward {sv_block}: loss {loss[0]:.6e} (oracle {g['loss']:.6e}), ||dg||/||g|| {rel:.2e}, "
          f"max|dg|/max|g| {rel_max:.2e}, vs oracle shift {rel_shift:.2e}, drift {drift[0]:.2e}")
    assert rel <= 1e-4 and rel_max <= 1e-4 and rel_shift <= 1e-4
    B = errmodel.state_bound(errmodel.plain_circuit_eps(circ))
    assert abs(loss[0] - g["loss"]) <= n * errmodel.z_bound(B)
    st.free()
    return got


@pytest.mark.parametrize("name", ["ring28", "ring28_small"])
def test_ring28_adjoint_vs_oracle(sv, name):
    """The differentiation workload at 28 qubits, random and small angles:
    the matrix-core backward (the autograd default at this size) and the
    per-gate backward against the oracle's 560 adjoint gradients and its
    parameter-shift values."""
    lam = torch.empty((1, 1 << 28), dtype=torch.complex64, device="cuda")
    g_mfma = _ring_check(name, svmod.ADJOINT_MFMA, lam)
    g_gate = _ring_check(name, 0, lam)
    assert np.max(np.abs(g_mfma - g_gate)) <= 1e-4 * np.max(np.abs(g_gate))


@pytest.mark.parametrize("name", ["ring28", "ring28_small"])
def test_ring28_adjoint_vs_gpu_parameter_shift(sv, name):
    """Parameter shift on the GPU, [L(t + pi/2) - L(t - pi/2)] / 2 with two
    plain forwards each, for 16 seeded parameters, against the matrix-core
    adjoint. Each shifted loss carries at most n (2 B + B^2) of rounding
    error; on the small-angle variant the gradients are O(0.1) and that
    bound is below 1e-4 relative, which is asserted too."""
    g = _golden(name)
    circ = C.WORKLOADS[name]()
    n = circ.n
    terms = C.z_sum_terms(n)
    st = svmod.State(n).reset().run(circ)
    _, grad, _ = st.adjoint_grad(circ, terms, block_qubits=svmod.ADJOINT_MFMA)
    adj = grad[0]
    which = np.random.default_rng(28).choice(circ.n_params, size=16, replace=False)
    B = errmodel.state_bound(errmodel.plain_circuit_eps(circ))
    lb = n * errmodel.z_bound(B)
    scale = float(np.max(np.abs(np.array(g["grad"]))))
    worst = 0.0
    for p in which:
        vals = []
        for sgn in (1.0, -1.0):
            prm = circ.params.copy()
            prm[p] += sgn * np.pi / 2
            st.reset().run(circ, prm)
            vals.append(float(np.sum(st.expval_z_all()[0][:n])))
        shift = 0.5 * (vals[0] - vals[1])
        assert abs(shift - adj[p]) <= lb
        assert abs(shift - g["grad"][p]) <= lb
        worst = max(worst, abs(shift - adj[p]))
    print(f"{name}: max |shift - adjoint| over 16 parameters {worst:.2e} (bound {lb:.2e}; max|g| {scale:.2e})")
    if name == "ring28_small":
        assert worst <= 1e-4 * scale
    st.free()
