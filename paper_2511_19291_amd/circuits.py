"""Seeded synthetic circuits: the only inputs the GPU path and the oracle share.

A circuit is plain data: qubit count, an ordered list of gates and a float64
parameter vector. This module draws angles and lays out gate lists; it holds
none of the simulation arithmetic (no matrices, no amplitudes), so both the
GPU library and the CPU oracle read the same circuit and compute everything
else independently.

Gate = (kind, targets, controls, param indices), the ordered pair (M, Q) of
the paper's Sec. 4.1.1 with M named by ``kind`` and Q = ``targets``; extra
control qubits make the controlled form of the gate. ``params`` indexes into
the circuit's parameter vector. Kinds:

  fixed, 1 target:  h x y z s sdg t tdg sx
  1 parameter:      rx ry rz p          (rotation exp(-i theta P / 2); p = phase)
  3 parameters:     u3                  (theta, phi, lambda)
  2 targets:        swap; rxx ryy rzz (1 parameter)

The paper's universal set is Pauli rotations plus CNOT (Sec. 3); CNOT is
``x`` with one control and CZ is ``z`` with one control.

Qubit q is bit q of the amplitude index (qubit 0 = least significant).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

FIXED_1Q = ("h", "x", "y", "z", "s", "sdg", "t", "tdg", "sx")
PARAM_1Q = ("rx", "ry", "rz", "p")
PARAM_3 = ("u3",)
FIXED_2Q = ("swap",)
PARAM_2Q = ("rxx", "ryy", "rzz")
ALL_KINDS = FIXED_1Q + PARAM_1Q + PARAM_3 + FIXED_2Q + PARAM_2Q

N_PARAMS = {k: 0 for k in FIXED_1Q + FIXED_2Q}
N_PARAMS.update({k: 1 for k in PARAM_1Q + PARAM_2Q})
N_PARAMS["u3"] = 3
N_TARGETS = {k: 1 for k in FIXED_1Q + PARAM_1Q + PARAM_3}
N_TARGETS.update({k: 2 for k in FIXED_2Q + PARAM_2Q})


@dataclass(frozen=True)
class Op:
    kind: str
    targets: Tuple[int, ...]
    controls: Tuple[int, ...] = ()
    params: Tuple[int, ...] = ()

    def qubits(self) -> Tuple[int, ...]:
        return tuple(self.targets) + tuple(self.controls)


@dataclass
class Circuit:
    n: int
    ops: List[Op]
    params: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # indices of params that are encoded inputs (features) rather than weights
    feature_idx: Tuple[int, ...] = ()
    name: str = ""

    @property
    def n_params(self) -> int:
        return int(len(self.params))

    def counts(self) -> dict:
        out: dict = {}
        for op in self.ops:
            key = ("c" * len(op.controls)) + op.kind
            out[key] = out.get(key, 0) + 1
        return out


def validate(c: Circuit) -> None:
    """Structural checks only (ranges, arity, disjoint wires)."""
    for op in c.ops:
        if op.kind not in ALL_KINDS:
            raise ValueError(f"unknown gate kind {op.kind!r}")
        if len(op.targets) != N_TARGETS[op.kind]:
            raise ValueError(f"{op.kind} takes {N_TARGETS[op.kind]} targets")
        if len(op.params) != N_PARAMS[op.kind]:
            raise ValueError(f"{op.kind} takes {N_PARAMS[op.kind]} params")
        wires = op.qubits()
        if len(set(wires)) != len(wires):
            raise ValueError(f"overlapping wires in {op}")
        if any(w < 0 or w >= c.n for w in wires):
            raise ValueError(f"wire out of range in {op} (n={c.n})")
        if any(p < 0 or p >= c.n_params for p in op.params):
            raise ValueError(f"param index out of range in {op}")


class _Builder:
    def __init__(self, n: int):
        self.n = n
        self.ops: List[Op] = []
        self.params: List[float] = []

    def gate(self, kind: str, targets: Sequence[int], controls: Sequence[int] = (),
             values: Sequence[float] = ()) -> None:
        idx = []
        for v in values:
            idx.append(len(self.params))
            self.params.append(float(v))
        self.ops.append(Op(kind, tuple(targets), tuple(controls), tuple(idx)))

    def build(self, name: str, feature_idx: Sequence[int] = ()) -> Circuit:
        c = Circuit(self.n, self.ops, np.asarray(self.params, dtype=np.float64),
                    tuple(feature_idx), name)
        validate(c)
        return c


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def hea_ladder(n: int = 12, layers: int = 4, seed: int = 1) -> Circuit:
    """Hardware-efficient ansatz: per layer RY on every qubit, RZ on every
    qubit, then a CNOT ladder q -> q+1 for q = 0..n-2 in increasing q.

    The ladder of CNOT + RY blocks is the paper's profiling ansatz (Sec. 5,
    Fig. 3); angles uniform in [0, 2 pi), drawn in gate order.
    """
    rng = _rng(seed)
    b = _Builder(n)
    for _ in range(layers):
        for q in range(n):
            b.gate("ry", [q], values=[rng.uniform(0.0, 2 * np.pi)])
        for q in range(n):
            b.gate("rz", [q], values=[rng.uniform(0.0, 2 * np.pi)])
        for q in range(n - 1):
            b.gate("x", [q + 1], [q])
    return b.build(f"hea_ladder_n{n}_l{layers}_s{seed}")


def brickwork_u3_cz(n: int = 30, layers: int = 20, seed: int = 2) -> Circuit:
    """Random brickwork: per layer a U3 on every qubit (theta, phi, lambda
    uniform in [0, 2 pi)), then CZ(q, q+1) for q = l mod 2, l mod 2 + 2, ...
    with q + 1 < n (layer l even: (0,1),(2,3)...; odd: (1,2),(3,4)...)."""
    rng = _rng(seed)
    b = _Builder(n)
    for layer in range(layers):
        for q in range(n):
            b.gate("u3", [q], values=rng.uniform(0.0, 2 * np.pi, size=3))
        for q in range(layer % 2, n - 1, 2):
            b.gate("z", [q + 1], [q])
    return b.build(f"brickwork_n{n}_l{layers}_s{seed}")


def rxry_ring(n: int = 28, layers: int = 10, seed: int = 5,
              small_angle: bool = False) -> Circuit:
    """Differentiation workload: per layer RX on every qubit, RY on every
    qubit, then a CNOT ring q -> (q+1) mod n for q = 0..n-1 (the ring of the
    paper's appendix example). 2 n layers parameters; angles uniform in
    [0, 2 pi), or in [-0.1, 0.1] for the small-angle variant."""
    rng = _rng(seed)
    lo, hi = (-0.1, 0.1) if small_angle else (0.0, 2 * np.pi)
    b = _Builder(n)
    for _ in range(layers):
        for q in range(n):
            b.gate("rx", [q], values=[rng.uniform(lo, hi)])
        for q in range(n):
            b.gate("ry", [q], values=[rng.uniform(lo, hi)])
        for q in range(n):
            b.gate("x", [(q + 1) % n], [q])
    return b.build(f"rxry_ring_n{n}_l{layers}_s{seed}{'_small' if small_angle else ''}")


def encoded_ansatz(n: int, layers: int, rng: np.random.Generator) -> Circuit:
    """Angle-encoded input (RY(x_q) on every qubit, features uniform in
    [-pi, pi], the GeneralEncoder of the paper's appendix example) followed by
    ``layers`` x [RY(theta) all q, RZ(theta) all q, CNOT ladder]."""
    b = _Builder(n)
    for q in range(n):
        b.gate("ry", [q], values=[rng.uniform(-np.pi, np.pi)])
    feats = tuple(range(n))
    for _ in range(layers):
        for q in range(n):
            b.gate("ry", [q], values=[rng.uniform(0.0, 2 * np.pi)])
        for q in range(n):
            b.gate("rz", [q], values=[rng.uniform(0.0, 2 * np.pi)])
        for q in range(n - 1):
            b.gate("x", [q + 1], [q])
    return b.build(f"encoded_ansatz_n{n}_l{layers}", feature_idx=feats)


def profiling_ladder(n: int, blocks: int = 3, batch: int = 16, seed: int = 6):
    """The paper's profiling workload (Sec. 5, Fig. 3; the appendix example):
    an RY(x_q) input encoding on every qubit, then ``blocks`` x [CNOT ring
    q -> (q + 1) mod n for q = 0..n-1, RY(theta_q) on every qubit]. The
    inputs x are trainable and differ per batch row (uniform in [0, pi/3) as
    in the example); the ansatz angles theta are shared by all rows (uniform in
    [0, 2 pi)). Draw order: theta in gate order, then x row by row.

    Returns (circuit, rows): the circuit's parameters are row 0's, and rows is
    the [batch, n + blocks n] parameter matrix (inputs first)."""
    rng = _rng(seed)
    b = _Builder(n)
    for q in range(n):
        b.gate("ry", [q], values=[0.0])
    for _ in range(blocks):
        for q in range(n):
            b.gate("x", [(q + 1) % n], [q])
        for q in range(n):
            b.gate("ry", [q], values=[0.0])
    theta = rng.uniform(0.0, 2 * np.pi, size=blocks * n)
    x = rng.uniform(0.0, np.pi / 3, size=(batch, n))
    rows = np.concatenate([x, np.broadcast_to(theta, (batch, blocks * n))], axis=1)
    circ = b.build(f"profiling_ladder_n{n}_b{blocks}", feature_idx=tuple(range(n)))
    circ.params = rows[0].copy()
    return circ, np.ascontiguousarray(rows)


def batch_workload(n_circuits: int = 256, nmin: int = 10, nmax: int = 20,
                   layers: int = 6, seed: int = 4) -> List[Circuit]:
    """Many uneven-size circuits: qubit counts uniform on {nmin..nmax}, each an
    encoded ansatz. Draw order: all qubit counts first, then each circuit's
    features and angles in gate order."""
    rng = _rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=n_circuits)
    return [encoded_ansatz(int(n), layers, rng) for n in ns]


def ghz(n: int) -> Circuit:
    """H on qubit 0 then a CNOT ladder: the GHZ state (|0..0> + |1..1>)/sqrt 2."""
    b = _Builder(n)
    b.gate("h", [0])
    for q in range(n - 1):
        b.gate("x", [q + 1], [q])
    return b.build(f"ghz_n{n}")


def basis_prep(n: int, j: int) -> List[Op]:
    """X gates that turn |0..0> into the basis state |j>."""
    return [Op("x", (q,)) for q in range(n) if (j >> q) & 1]


def qft(n: int, j: int = 0, swaps: bool = True) -> Circuit:
    """Textbook QFT network on the basis state |j>: for the most significant
    qubit downwards, H then controlled phases CP(pi / 2^m), then a qubit
    reversal by swaps. Acting on |j> it yields
    sum_k exp(2 pi i j k / 2^n) |k> / sqrt(2^n)."""
    b = _Builder(n)
    b.ops.extend(basis_prep(n, j))
    for i in reversed(range(n)):
        b.gate("h", [i])
        for m, c in enumerate(reversed(range(i)), start=1):
            b.gate("p", [i], [c], values=[np.pi / 2 ** m])
    if swaps:
        for q in range(n // 2):
            b.gate("swap", [q, n - 1 - q])
    return b.build(f"qft_n{n}_j{j}")


def random_circuit(n: int, n_gates: int, seed: int, kinds: Sequence[str] = ALL_KINDS,
                   max_controls: int = 2) -> Circuit:
    """Random mix of every gate kind, with random targets/controls, for
    coverage of kernel variants (every target position, control pattern and
    kind)."""
    rng = _rng(seed)
    b = _Builder(n)
    for _ in range(n_gates):
        kind = str(rng.choice(list(kinds)))
        nt = N_TARGETS[kind]
        if nt > n:
            continue
        nc = int(rng.integers(0, min(max_controls, n - nt) + 1))
        wires = rng.permutation(n)[: nt + nc]
        vals = rng.uniform(0.0, 2 * np.pi, size=N_PARAMS[kind])
        b.gate(kind, [int(w) for w in wires[:nt]], [int(w) for w in wires[nt:]], vals)
    return b.build(f"random_n{n}_g{n_gates}_s{seed}")


def inverse(c: Circuit) -> Circuit:
    """The gate list reversed with each gate replaced by its inverse, written
    with the same kinds: rotations negate their angle, u3(t,f,l)^-1 =
    u3(-t,-l,-f), s <-> sdg, t <-> tdg; self-inverse kinds stay. sx is not
    supported (its inverse is not a listed kind)."""
    b = _Builder(c.n)
    params = list(c.params)
    for op in reversed(c.ops):
        k = op.kind
        if k in ("h", "x", "y", "z", "swap"):
            b.ops.append(Op(k, op.targets, op.controls, ()))
        elif k in ("s", "sdg", "t", "tdg"):
            swap = {"s": "sdg", "sdg": "s", "t": "tdg", "tdg": "t"}[k]
            b.ops.append(Op(swap, op.targets, op.controls, ()))
        elif k in PARAM_1Q + PARAM_2Q:
            b.gate(k, op.targets, op.controls, [-params[op.params[0]]])
        elif k == "u3":
            t, f, lam = (params[i] for i in op.params)
            b.gate("u3", op.targets, op.controls, [-t, -lam, -f])
        else:
            raise ValueError(f"no inverse written for kind {k!r}")
    return b.build(c.name + "_inv")


# Observables: a Pauli term is (coeff, x_mask, z_mask), bit q of x_mask set
# for X or Y on qubit q and bit q of z_mask set for Z or Y. (Y = i X Z.)

def pauli_term(coeff: float, spec: str) -> Tuple[float, int, int]:
    """Parse e.g. "X0 Y3 Z5" into (coeff, x_mask, z_mask)."""
    xm = zm = 0
    for tok in spec.split():
        p, q = tok[0].upper(), int(tok[1:])
        if p not in "XYZ":
            raise ValueError(f"bad Pauli {tok!r}")
        if p in "XY":
            xm |= 1 << q
        if p in "YZ":
            zm |= 1 << q
    return (float(coeff), xm, zm)


def z_sum_terms(n: int) -> List[Tuple[float, int, int]]:
    """sum_i Z_i as a term list."""
    return [(1.0, 0, 1 << i) for i in range(n)]


# Named workloads with their sizes (the five measured configurations).
WORKLOADS = {
    "hea12": lambda: hea_ladder(12, 4, 1),
    "brickwork30": lambda: brickwork_u3_cz(30, 20, 2),
    "brickwork24": lambda: brickwork_u3_cz(24, 20, 2),
    "fused32": lambda: brickwork_u3_cz(32, 20, 3),
    "fused24": lambda: brickwork_u3_cz(24, 20, 3),
    "ring28": lambda: rxry_ring(28, 10, 5),
    "ring28_small": lambda: rxry_ring(28, 10, 55, small_angle=True),
    "ring14": lambda: rxry_ring(14, 10, 5),
}
