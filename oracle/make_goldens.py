"""Write the stored expected values of the full-size parity tests -- TEST
INFRASTRUCTURE.

    python oracle/make_goldens.py [brickwork30] [batch256] [profiling24] [ring28] [ring28_small]

Every value comes from the complex128 oracle in this package, run on the
seeded circuits of ``paper_2511_19291_amd/circuits.py`` (plain data: gate
lists and angles, no arithmetic). Nothing here reads the GPU library. The
outputs go to ``tests/golden/<name>.json``; each file records the circuit,
the oracle routines used and the wall time they took.

brickwork30    30-qubit brickwork (20 layers of U3 + CZ on alternating pairs,
               seed 2; the benchmark step): <Z_i> for every qubit, <sum Z_i>,
               the norm, and 1024 amplitudes at seeded indices (plus the first
               and the last index). The complex128 state is 16 GiB.
batch256       all 256 circuits of the batching workload (10..20 qubits, seed
               4): <Z_i> for every qubit of every circuit.
profiling24    the paper's profiling ladder at 24 qubits, batch 16 (seed 7),
               with a seeded weight matrix c[r, i]: per row the loss
               sum_i c[r, i] <Z_i> and its gradient in every parameter
               (inputs and angles) by the oracle's adjoint (Sec. 4.4).
ring28         the 28-qubit RX/RY + CNOT-ring workload (seed 5; the small-angle
ring28_small   variant seed 55): the loss <sum Z_i>, all 560 gradients by the
               oracle's adjoint, and four of them again by the parameter-shift
               rule (the two routes must agree to 1e-9 before anything is
               written).
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2511_19291_amd import circuits as C  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")


def _log(msg: str) -> None:
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _write(name: str, obj: dict) -> None:
    path = os.path.join(GOLDEN, name + ".json")
    with open(path + ".tmp", "w") as f:
        json.dump(obj, f, indent=1)
        f.write("\n")
    os.replace(path + ".tmp", path)
    _log(f"wrote {path}")


def _zterms(n, c=None):
    return [(1.0 if c is None else float(c[i]), 0, 1 << i) for i in range(n)]


def sample_indices(n: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct amplitude indices: 0, 2^n - 1 and ``count`` seeded
    draws (PCG64). The tests read the indices from the file."""
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = set(int(v) for v in rng.integers(0, 1 << n, size=count))
    idx.update((0, (1 << n) - 1))
    return np.array(sorted(idx), dtype=np.int64)


def brickwork30() -> None:
    circ = C.WORKLOADS["brickwork30"]()
    n = circ.n
    t0 = time.time()
    psi = oracle.basis_state(n, 0)
    for i, op in enumerate(circ.ops):
        oracle.apply_op(psi, n, op, circ.params)
        if i % 50 == 0:
            _log(f"brickwork30 gate {i}/{len(circ.ops)}")
    t_run = time.time() - t0
    z, norm2 = oracle.expval_z_all(psi, n)
    idx = sample_indices(n, 1024, 30)
    amps = psi[idx]
    _write("brickwork30", {
        "source": "oracle.run + oracle.expval_z_all on circuits.brickwork_u3_cz(30, 20, 2) "
                  "(Alg. 1 per gate, complex128; Sec. 2.2.1 Z measurement)",
        "command": "python oracle/make_goldens.py brickwork30",
        "circuit": circ.name, "n": n, "n_gates": len(circ.ops),
        "oracle_seconds": round(t_run, 1),
        "expval_z": [float(v) for v in z],
        "sum_z": float(np.sum(z)),
        "norm2": norm2,
        "sample_seed": 30,
        "amp_index": [int(v) for v in idx],
        "amp_re": [float(v) for v in amps.real],
        "amp_im": [float(v) for v in amps.imag],
    })


def batch256() -> None:
    circuits = C.batch_workload(256, 10, 20, 6, 4)
    t0 = time.time()
    zs = []
    for c in circuits:
        z, _ = oracle.expval_z_all(oracle.run(c), c.n)
        zs.append([float(v) for v in z])
    _write("batch256", {
        "source": "oracle.run + oracle.expval_z_all on every circuit of "
                  "circuits.batch_workload(256, 10, 20, 6, 4) (Alg. 1, complex128)",
        "command": "python oracle/make_goldens.py batch256",
        "n_qubits": [c.n for c in circuits],
        "oracle_seconds": round(time.time() - t0, 1),
        "expval_z": zs,
    })


def profiling24() -> None:
    n, B = 24, 16
    circ, rows = C.profiling_ladder(n, 3, B, seed=7)
    coeff = np.random.Generator(np.random.PCG64(24)).normal(size=(B, n))
    t0 = time.time()
    losses, grads = [], []
    for r in range(B):
        L, g, drift = oracle.grad_adjoint(circ, _zterms(n, coeff[r]), params=rows[r])
        assert drift < 1e-10, drift
        losses.append(L)
        grads.append([float(v) for v in g])
        _log(f"profiling24 row {r}")
    _write("profiling24", {
        "source": "oracle.grad_adjoint (Sec. 4.4, recompute by inverse, complex128) per row of "
                  "circuits.profiling_ladder(24, 3, 16, seed=7) with observable sum_i c[r,i] Z_i",
        "command": "python oracle/make_goldens.py profiling24",
        "circuit": circ.name, "n": n, "batch": B,
        "coeff_seed": 24,
        "coeff": [[float(v) for v in row] for row in coeff],
        "oracle_seconds": round(time.time() - t0, 1),
        "loss": [float(v) for v in losses],
        "grad": grads,
    })


def _shift_grads(circ, terms, which):
    """Parameter shift [L(t + pi/2) - L(t - pi/2)] / 2 for the given
    parameters, each used by exactly one gate; the state before that gate is
    shared by both shifts (a running prefix, advanced in gate order)."""
    n = circ.n
    params = np.asarray(circ.params, dtype=np.float64)
    gate_of = {}
    for gi, op in enumerate(circ.ops):
        for p in op.params:
            assert p not in gate_of, "parameter used by more than one gate"
            gate_of[p] = gi
    out = {}
    prefix = oracle.basis_state(n, 0)
    done = 0
    for p in sorted(which, key=lambda q: gate_of[q]):
        g = gate_of[p]
        for op in circ.ops[done:g]:
            oracle.apply_op(prefix, n, op, params)
        done = g
        vals = []
        for sgn in (+1.0, -1.0):
            shifted = params.copy()
            shifted[p] += sgn * np.pi / 2
            psi = prefix.copy()
            for op in circ.ops[g:]:
                oracle.apply_op(psi, n, op, shifted)
            vals.append(oracle.expval_terms(psi, n, terms))
            del psi
        out[p] = 0.5 * (vals[0] - vals[1])
        _log(f"{circ.name}: shift gradient of parameter {p} = {out[p]:.6e}")
    return out


def ring(name: str) -> None:
    circ = C.WORKLOADS[name]()
    n = circ.n
    terms = _zterms(n)
    t0 = time.time()
    L, g, drift = oracle.grad_adjoint(circ, terms)
    t_adj = time.time() - t0
    _log(f"{name}: adjoint done in {t_adj:.0f} s, loss {L:.6e}, drift {drift:.2e}")
    assert drift < 1e-10, drift
    which = (0, 200, 401, 559)
    t1 = time.time()
    shift = _shift_grads(circ, terms, which)
    t_shift = time.time() - t1
    scale = max(1e-12, float(np.max(np.abs(g))))
    for p, v in shift.items():
        assert abs(v - g[p]) <= 1e-9 * max(1.0, scale), (p, v, g[p])
    _write(name, {
        "source": f"oracle.grad_adjoint (Sec. 4.4) on circuits.WORKLOADS[{name!r}] with loss <sum Z_i>, "
                  "and the parameter-shift rule for four parameters (running prefix, complex128)",
        "command": f"python oracle/make_goldens.py {name}",
        "circuit": circ.name, "n": n, "n_params": circ.n_params,
        "oracle_seconds_adjoint": round(t_adj, 1),
        "oracle_seconds_shift": round(t_shift, 1),
        "loss": float(L),
        "drift": float(drift),
        "grad": [float(v) for v in g],
        "shift_params": [int(p) for p in which],
        "shift_grad": [float(shift[p]) for p in which],
    })


JOBS = {
    "brickwork30": brickwork30,
    "batch256": batch256,
    "profiling24": profiling24,
    "ring28": lambda: ring("ring28"),
    "ring28_small": lambda: ring("ring28_small"),
}


def main(argv) -> int:
    names = argv or list(JOBS)
    for nm in names:
        if nm not in JOBS:
            print(f"unknown golden {nm!r}; choose from {sorted(JOBS)}", file=sys.stderr)
            return 2
    for nm in names:
        _log(f"start {nm}")
        JOBS[nm]()
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
