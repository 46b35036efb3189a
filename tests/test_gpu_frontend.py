"""The front end on the GPU: the appendix example's training loop end to end
(encoder, CNOT ring, trainable RY modules, measure_allZ, Adam), checked
against the oracle, and the three generated forms of every gate against
each other and the oracle."""

import numpy as np
import pytest
import torch

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import frontend as F

pytestmark = pytest.mark.gpu


def _listing(nq):
    enc = F.GeneralEncoder([{"func": "ry", "wires": [i], "input_idx": [i]} for i in range(nq)])
    base = [enc]
    for _ in range(3):
        base = base + [F.CX(wires=[i, (i + 1) % nq]) for i in range(nq)] + [F.RY(wires=[i]) for i in range(nq)]
    return F.InvertibleUnitary(base)


def _oracle_listing(mod, x_row, nq):
    """The same circuit written directly for the oracle: parameters are the
    row's inputs, then every RY module's angle in order."""
    b = C._Builder(nq)
    for i in range(nq):
        b.gate("ry", [i], values=[float(x_row[i])])
    for m in mod.layers[1:]:
        kind, nc, nt, npar = F.GATE_SCHEMA[m.name]
        vals = [float(v) for v in m.params.detach()] if npar else []
        b.gate(kind, m.wires[nc:], m.wires[:nc], values=vals)
    return b.build("listing")


def test_listing_training_loop_vs_oracle(sv):
    torch.manual_seed(0)
    nq, batch = 6, 4
    qdev = F.QuantumDevice(nq, bsz=batch, device="cuda", world_sz=1, invertible=True)
    mod = _listing(nq)
    mod.train()
    x = torch.nn.Parameter(torch.rand([batch, nq], device="cuda", dtype=torch.float64) * torch.pi / 3)

    def fun(inp):
        qdev.reset_states()
        mod(qdev, inp)
        return F.measure_allZ(qdev, shots=0, training=True)

    # first step: outputs and gradients (inputs and ansatz angles) vs the oracle
    out = fun(x)
    loss = out.abs().sum()
    loss.backward()
    xs = x.detach().cpu().numpy()
    ry_mods = [m for m in mod.layers[1:] if m.name == "ry"]
    g_theta = np.zeros(len(ry_mods))
    for r in range(batch):
        circ = _oracle_listing(mod, xs[r], nq)
        z, _ = oracle.expval_z_all(oracle.run(circ), nq)
        np.testing.assert_allclose(out[r].detach().cpu().numpy(), z[:nq], atol=2e-6)
        w = [(float(np.sign(z[i])), 0, 1 << i) for i in range(nq)]
        g = oracle.grad_param_shift(circ, w)
        np.testing.assert_allclose(x.grad[r].cpu().numpy(), g[:nq], atol=1e-5)
        g_theta += g[nq:]
    got_theta = np.array([float(m.params.grad[0]) for m in ry_mods])
    np.testing.assert_allclose(got_theta, g_theta, atol=1e-5 * batch)
    # the loop of the example: the loss goes down
    opt = torch.optim.Adam([x] + list(mod.parameters()), lr=0.05)
    losses = []
    for _ in range(10):
        opt.zero_grad()
        loss = fun(x).abs().sum()
        losses.append(loss.item())
        loss.backward()
        opt.step()
    assert losses[-1] < losses[0]


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
