"""Python front end in the style of the paper's listings (Sec. 3, Appendix A).

Gates are defined once, in ``GATE_SCHEMA``, and three forms are generated
from that table programmatically (the paper's "code parsimony" principle,
Sec. 3):

* functional:   ``functional.ry(qdev, wires=[0], params=theta)``
* device method: ``qdev.ry(wires=[0], params=theta)``
* module:       ``RY(wires=[0])`` -- an ``nn.Module`` owning its trainable
  angles, applied as ``RY(wires=[0])(qdev)``.

plus ``GeneralEncoder`` (input features as rotation angles, one column per
gate), ``InvertibleUnitary`` (a list of modules whose backward un-applies the
gates, Sec. 4.4) and ``measure_allZ`` (exact, or with shots: exact draws, or
the differentiable Gaussian estimate in training).

Execution model: a ``QuantumDevice`` records the gates applied to it since
its last ``reset_states()`` together with their angle tensors (a scalar
shared by every batch row, or one value per row). ``measure_allZ`` turns the
record into one circuit and one [batch, n_params] parameter matrix (built
with torch ops, so gradients flow back to every angle tensor), and runs it
through the GPU library: forward sweeps, <Z_i> per row, and on backward the
adjoint method, which recomputes each layer's input by un-applying the gates
instead of storing it. Wires follow the listings: for controlled gates the
leading wires are the controls (``CX(wires=[c, t])``).

One GPU only: ``world_sz`` other than 1 is refused (the sharded state of the
paper's Sec. 4.2 is not part of this library).
"""

from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import circuits as C
from . import sv
from .autograd import ExpvalZ, GaussianExpvalZ, default_block_qubits, default_fuse

# name -> (kind, number of controls, number of targets, number of angles)
GATE_SCHEMA: Dict[str, Tuple[str, int, int, int]] = {
    "h": ("h", 0, 1, 0), "x": ("x", 0, 1, 0), "y": ("y", 0, 1, 0), "z": ("z", 0, 1, 0),
    "s": ("s", 0, 1, 0), "sdg": ("sdg", 0, 1, 0), "t": ("t", 0, 1, 0), "tdg": ("tdg", 0, 1, 0),
    "sx": ("sx", 0, 1, 0),
    "rx": ("rx", 0, 1, 1), "ry": ("ry", 0, 1, 1), "rz": ("rz", 0, 1, 1), "p": ("p", 0, 1, 1),
    "u3": ("u3", 0, 1, 3),
    "swap": ("swap", 0, 2, 0), "rxx": ("rxx", 0, 2, 1), "ryy": ("ryy", 0, 2, 1), "rzz": ("rzz", 0, 2, 1),
    "cx": ("x", 1, 1, 0), "cnot": ("x", 1, 1, 0), "cy": ("y", 1, 1, 0), "cz": ("z", 1, 1, 0),
    "ch": ("h", 1, 1, 0),
    "crx": ("rx", 1, 1, 1), "cry": ("ry", 1, 1, 1), "crz": ("rz", 1, 1, 1), "cp": ("p", 1, 1, 1),
    "cu3": ("u3", 1, 1, 3),
    "ccx": ("x", 2, 1, 0), "toffoli": ("x", 2, 1, 0), "cswap": ("swap", 1, 2, 0),
}


class QuantumDevice:
    """A batch of ``bsz`` states of ``n_wires`` qubits on one GPU, and the
    record of the gates applied since the last ``reset_states()``."""

    def __init__(self, n_wires: int, bsz: int = 1, device="cuda", world_sz: int = 1, invertible: bool = True):
        if world_sz != 1:
            raise ValueError("this library keeps the state on one GPU (world_sz must be 1)")
        if not invertible:
            raise ValueError("only the invertible device is provided: the backward un-applies the gates")
        self.n_wires = n_wires
        self.bsz = bsz
        self.device = torch.device(device)
        self.state = sv.State(n_wires, bsz, device=self.device)
        self.reset_states()

    def reset_states(self) -> None:
        """Every row back to |0..0>; the gate record is cleared."""
        self._ops: List[C.Op] = []
        self._angles: List[torch.Tensor] = []       # each [bsz] float64 (per row or broadcast)

    def apply(self, name: str, wires: Sequence[int], params=None) -> None:
        kind, nc, nt, npar = GATE_SCHEMA[name]
        wires = [int(w) for w in wires]
        if len(wires) != nc + nt:
            raise ValueError(f"{name} takes {nc + nt} wires, got {len(wires)}")
        idx = []
        if npar:
            if params is None:
                raise ValueError(f"{name} takes {npar} angle(s)")
            p = torch.as_tensor(params, dtype=torch.float64)
            if p.dim() == 0:
                p = p.reshape(1)
            if p.dim() == 1 and npar == 1 and p.numel() == self.bsz and self.bsz > 1:
                cols = [p]                                   # one angle per row
            elif p.dim() == 2:
                if p.shape != (self.bsz, npar):
                    raise ValueError(f"{name}: per-row angles must be [bsz, {npar}]")
                cols = [p[:, j] for j in range(npar)]
            else:
                if p.numel() != npar:
                    raise ValueError(f"{name} takes {npar} angle(s), got {p.numel()}")
                cols = [p.reshape(npar)[j].expand(self.bsz) for j in range(npar)]
            for c in cols:
                idx.append(len(self._angles))
                self._angles.append(c.to(torch.float64))
        self._ops.append(C.Op(kind, tuple(wires[nc:]), tuple(wires[:nc]), tuple(idx)))

    # the recorded circuit and its [bsz, n_params] angle matrix
    def _program(self):
        circ = C.Circuit(self.n_wires, list(self._ops), np.zeros(len(self._angles)), name="recorded")
        if self._angles:
            mat = torch.stack([a.cpu() if a.device.type != "cpu" else a for a in self._angles], dim=1)
        else:
            mat = torch.zeros((self.bsz, 0), dtype=torch.float64)
        return circ, mat

    def __getattr__(self, name):
        # device-method forms: qdev.rx(wires=[0], params=theta)
        if name in GATE_SCHEMA:
            return lambda wires, params=None: self.apply(name, wires, params)
        raise AttributeError(name)


class _Functional:
    """Functional forms generated from the schema: functional.ry(qdev, wires, params)."""

    def __init__(self):
        for name in GATE_SCHEMA:
            setattr(self, name, self._make(name))

    @staticmethod
    def _make(name):
        def f(qdev: QuantumDevice, wires: Sequence[int], params=None) -> None:
            qdev.apply(name, wires, params)
        f.__name__ = name
        f.__doc__ = f"Apply {name} ({GATE_SCHEMA[name][0]}, {GATE_SCHEMA[name][1]} control(s)) to qdev."
        return f


functional = _Functional()


class GateModule(torch.nn.Module):
    """Module form of one schema entry; trainable angles are nn.Parameters
    (initialised uniform in [0, 2 pi) unless given)."""

    name = ""

    def __init__(self, wires: Sequence[int], trainable: bool = True, init_params=None):
        super().__init__()
        self.wires = [int(w) for w in wires]
        npar = GATE_SCHEMA[self.name][3]
        if npar:
            init = torch.rand(npar, dtype=torch.float64) * 2 * np.pi if init_params is None \
                else torch.as_tensor(init_params, dtype=torch.float64).reshape(npar)
            if trainable:
                self.params = torch.nn.Parameter(init.clone())
            else:
                self.register_buffer("params", init.clone())
        else:
            self.params = None

    def forward(self, qdev: QuantumDevice) -> None:
        qdev.apply(self.name, self.wires, self.params)


def _module_class(name: str):
    return type(name.upper(), (GateModule,), {"name": name, "__doc__": f"Module form of {name}."})


# module forms: RX, RY, CX, ... (upper-case names), generated from the schema
MODULES = {name: _module_class(name) for name in GATE_SCHEMA}
globals().update({cls.__name__: cls for cls in MODULES.values()})


class GeneralEncoder(torch.nn.Module):
    """Input features as gate angles (the appendix example's encoder): each
    entry {'func': name, 'wires': [...], 'input_idx': [...]} applies the gate
    with the listed columns of the input [bsz, n_features] as its angles."""

    def __init__(self, func_list: Sequence[dict]):
        super().__init__()
        self.func_list = [dict(f) for f in func_list]

    def forward(self, qdev: QuantumDevice, x: torch.Tensor) -> None:
        for f in self.func_list:
            cols = x[:, list(f["input_idx"])]
            qdev.apply(f["func"], f["wires"], cols if cols.shape[1] > 1 else cols[:, 0])


class InvertibleUnitary(torch.nn.Module):
    """A sequence of modules (encoders take the input) applied in order. Its
    gradient is computed by the adjoint method, which un-applies the gates
    from the final state (Sec. 4.4) rather than storing layer inputs."""

    def __init__(self, modules: Sequence[torch.nn.Module]):
        super().__init__()
        self.layers = torch.nn.ModuleList(modules)

    def forward(self, qdev: QuantumDevice, x: Optional[torch.Tensor] = None) -> None:
        for m in self.layers:
            if isinstance(m, GeneralEncoder):
                if x is None:
                    raise ValueError("an encoder needs the input")
                m(qdev, x)
            else:
                m(qdev)


def ring_ansatz(n_wires: int, layers: int, rotation: str = "ry", encoding: str = "ry") -> InvertibleUnitary:
    """A layered model of the ladder family the paper profiles (Sec. 5,
    Fig. 3; Appendix A): feature i encoded as the angle of an ``encoding``
    gate on wire i, then ``layers`` x [a trainable ``rotation`` on every
    wire, a CNOT ring i -> (i + 1) mod n]."""
    mods: list = [GeneralEncoder([{"func": encoding, "wires": [w], "input_idx": [w]} for w in range(n_wires)])]
    rot, cx = MODULES[rotation], MODULES["cx"]
    for _ in range(layers):
        mods.extend(rot(wires=[w]) for w in range(n_wires))
        mods.extend(cx(wires=[w, (w + 1) % n_wires]) for w in range(n_wires))
    return InvertibleUnitary(mods)


def measure_allZ(qdev: QuantumDevice, shots: int = 0, training: bool = True, generator=None) -> torch.Tensor:
    """<Z_i> of every wire for every row, [bsz, n_wires].

    shots = 0: exact expectations (Sec. 2.2.1), differentiable through the
    adjoint backward. shots > 0 and training: the Gaussian shot-noise
    estimate (Sec. 4.3.2), differentiable by reparameterisation (normals
    drawn here, with ``generator`` if given, and held fixed for the
    backward). shots > 0 and not training: estimates from exact shot sampling
    (Sec. 4.3.1: inverse-CDF draws on the GPU), not differentiable."""
    circ, mat = qdev._program()
    mat = mat.to(torch.float64)
    if shots == 0:
        z = ExpvalZ.apply(mat, circ, qdev.state, default_block_qubits(circ), default_fuse(circ, qdev.bsz))
        return z.to(qdev.device) if qdev.device.type == "cuda" else z
    if training:
        normals = torch.randn((qdev.bsz, 1 << qdev.n_wires), dtype=torch.float64, device=qdev.device,
                              generator=generator)
        z = GaussianExpvalZ.apply(mat, circ, qdev.state, normals, float(shots), default_block_qubits(circ),
                                  default_fuse(circ, qdev.bsz))
        return z.to(qdev.device)
    with torch.no_grad():
        p = mat.detach().numpy()
        qdev.state.reset()
        qdev.state.run(circ, params=p if qdev.bsz > 1 else p[0])
        out = torch.empty((qdev.bsz, qdev.n_wires), dtype=torch.float64, device=qdev.device)
        for r in range(qdev.bsz):
            u = torch.rand(int(shots), dtype=torch.float64, device=qdev.device, generator=generator)
            idx = qdev.state.sample_exact(u, row=r)
            out[r] = qdev.state.sample_z_estimate(idx)
        return out
