"""The front end on the GPU: a layered model built with the front end
(encoder, trainable rotations, CNOT rings, measure_allZ) trained on its
inputs and angles, checked against the oracle, and the three generated forms
of every gate against each other and the oracle. The model family and the
API names are those of the paper's Appendix A."""

import numpy as np
import pytest
import torch

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import frontend as F

pytestmark = pytest.mark.gpu


def _oracle_circuit(mod, x_row, nq):
    """The model written directly for the oracle: parameters are the row's
    inputs, then every trainable module's angle in order."""
    b = C._Builder(nq)
    for f in mod.layers[0].func_list:
        b.gate(f["func"], f["wires"], values=[float(x_row[f["input_idx"][0]])])
    for m in mod.layers[1:]:
        kind, nc, nt, npar = F.GATE_SCHEMA[m.name]
        vals = [float(v) for v in m.params.detach()] if npar else []
        b.gate(kind, m.wires[nc:], m.wires[:nc], values=vals)
    return b.build("front_end_model")


def _squared_error(qdev, mod, x, target):
    qdev.reset_states()
    mod(qdev, x)
    z = F.measure_allZ(qdev, shots=0, training=True)
    return z, ((z - target) ** 2).sum()


@pytest.mark.parametrize("rotation", ["ry", "rx"])
def test_model_gradients_and_training_vs_oracle(sv, rotation):
    gen = torch.Generator().manual_seed(3)
    nq, batch, layers = 5, 3, 2
    qdev = F.QuantumDevice(nq, bsz=batch, device="cuda")
    mod = F.ring_ansatz(nq, layers, rotation=rotation)
    mod.train()
    x = torch.nn.Parameter((torch.rand((batch, nq), generator=gen, dtype=torch.float64) * 2 - 1).cuda())
    target = torch.linspace(-0.5, 0.5, nq, dtype=torch.float64, device="cuda")
    z, loss = _squared_error(qdev, mod, x, target)
    loss.backward()
    # outputs and gradients (inputs and every trainable angle) vs the oracle
    xs = x.detach().cpu().numpy()
    rots = [m for m in mod.layers[1:] if m.name == rotation]
    g_theta = np.zeros(len(rots))
    t = target.cpu().numpy()
    for r in range(batch):
        circ = _oracle_circuit(mod, xs[r], nq)
        zr, _ = oracle.expval_z_all(oracle.run(circ), nq)
        np.testing.assert_allclose(z[r].detach().cpu().numpy(), zr[:nq], atol=2e-6)
        w = [(2.0 * float(zr[i] - t[i]), 0, 1 << i) for i in range(nq)]   # d loss / d <Z_i>
        g = oracle.grad_param_shift(circ, w)
        np.testing.assert_allclose(x.grad[r].cpu().numpy(), g[:nq], atol=1e-5)
        g_theta += g[nq:]
    got_theta = np.array([float(m.params.grad[0]) for m in rots])
    np.testing.assert_allclose(got_theta, g_theta, atol=1e-5 * batch)
    # a few optimiser steps on inputs and angles lower the loss
    opt = torch.optim.SGD([x] + list(mod.parameters()), lr=0.1)
    first = loss.item()
    for _ in range(8):
        opt.zero_grad()
        _, loss = _squared_error(qdev, mod, x, target)
        loss.backward()
        opt.step()
    assert loss.item() < first


def test_three_forms_agree(sv):
    """Every schema entry through its functional, method and module form on
    a random state: identical states, equal to the oracle's."""
    nq = 5
    rng = np.random.default_rng(3)
    names = list(F.GATE_SCHEMA)
    plan = []
    for name in names:
        kind, nc, nt, npar = F.GATE_SCHEMA[name]
        wires = [int(w) for w in rng.permutation(nq)[: nc + nt]]
        plan.append((name, wires, rng.uniform(0, 2 * np.pi, size=npar)))
    outs = []
    for form in ("functional", "method", "module"):
        qdev = F.QuantumDevice(nq, bsz=1)
        for name, wires, vals in plan:
            p = torch.tensor(vals) if len(vals) else None
            if form == "functional":
                getattr(F.functional, name)(qdev, wires, p)
            elif form == "method":
                getattr(qdev, name)(wires, p)
            else:
                F.MODULES[name](wires, init_params=vals if len(vals) else None)(qdev)
        outs.append(F.measure_allZ(qdev).detach().cpu().numpy())
        st = qdev.state.to_numpy()[0]
        outs.append(st)
    b = C._Builder(nq)
    for name, wires, vals in plan:
        kind, nc, nt, npar = F.GATE_SCHEMA[name]
        b.gate(kind, wires[nc:], wires[:nc], values=list(vals))
    ref = oracle.run(b.build("forms"))
    for st in outs[1::2]:
        np.testing.assert_allclose(st, ref, atol=1e-5)
    np.testing.assert_allclose(outs[0], outs[2], atol=1e-7)
    np.testing.assert_allclose(outs[0], outs[4], atol=1e-7)


def test_shot_estimates_and_refusals(sv):
    nq = 4
    qdev = F.QuantumDevice(nq, bsz=2)
    x = torch.tensor([[0.3, 1.1, 2.0, 0.7], [1.5, 0.2, 0.9, 2.8]], dtype=torch.float64)
    enc = F.GeneralEncoder([{"func": "ry", "wires": [i], "input_idx": [i]} for i in range(nq)])
    enc(qdev, x)
    exact = F.measure_allZ(qdev).detach().cpu().numpy()
    np.testing.assert_allclose(exact, np.cos(x.numpy()), atol=1e-6)
    est = F.measure_allZ(qdev, shots=200_000, training=False).cpu().numpy()
    assert np.max(np.abs(est - exact)) < 5 * 1 / np.sqrt(200_000) + 1e-9
    # training: the Gaussian estimate, differentiable in the inputs
    xg = x.clone().requires_grad_(True)
    qdev.reset_states()
    enc(qdev, xg)
    gen = torch.Generator(device="cuda").manual_seed(3)
    noisy = F.measure_allZ(qdev, shots=200_000, training=True, generator=gen)
    assert np.max(np.abs(noisy.detach().cpu().numpy() - exact)) < 5 * 1 / np.sqrt(200_000) + 1e-9
    noisy.sum().backward()
    assert xg.grad is not None and np.all(np.isfinite(xg.grad.numpy()))
    # d<Z_i>/dx_i = -sin(x_i) for the noise-free part; the noise adds O(1/sqrt(shots))
    np.testing.assert_allclose(xg.grad.numpy(), -np.sin(x.numpy()), atol=0.05)
    with pytest.raises(ValueError):
        F.QuantumDevice(nq, world_sz=2)
