"""Rounding-error bounds the GPU parity tests assert (test infrastructure).

Every sweep g over the state (one gate, one fused block, one register
phase) computes y = M x for each group of D = 2^k amplitudes. Each real
output component is a dot product of L = 2 D real terms m * x. Let eps_g
bound the relative error of every term's contribution (operand
representation, product, accumulation):

* a plain FP32 gate sweep (k <= 2): the matrix rounded to FP32 (u), the
  product and an L-term FP32 accumulation in any order (L u):
  eps = (L + 1) u, u = 2^-24;
* an FP32 matrix-core block on k qubits, same count; in the three-real-
  product (Gauss) form the operand sums (a + b), (c + d), (d - c) are
  rounded too and |a| + |b| <= sqrt 2 |a + i b|: eps = sqrt 2 (L + 3) u;
* a BF16x3 block: each FP32 operand a = a_hi + a_lo + r with a_hi =
  bf16(a), a_lo = bf16(a - a_hi), so |r| <= 2^-8 |a - a_hi| <= 2^-16 |a|
  (bf16 keeps 8 significant bits); the product is formed as
  a_hi b_hi + a_hi b_lo + a_lo b_hi (each exact in FP32), dropping
  a_lo b_lo (<= 2^-16 |a b|): 3 * 2^-16 from the split, plus an FP32
  accumulation of 3 L exact products: eps = 3 * 2^-16 + (3 L + 1) u.

Model (probabilistic rounding-error analysis in the style of Higham and
Mary, SIAM J. Sci. Comput. 41 (2019)): the individual errors are
independent, mean zero and bounded by eps_g |m x|, so by Hoeffding's
inequality and because the columns of a unitary M have unit norm, the
error a sweep adds to the state has norm about sqrt 2 eps_g ||x|| (sqrt 2:
real and imaginary parts), and errors of different sweeps add in
quadrature (a unitary sweep carries earlier errors along unchanged in
norm). With a safety factor K = 4:

    ||dpsi||_2 <= B = K sqrt(sum_g 2 eps_g^2)

and, rigorously given ||dpsi|| <= B and ||psi|| = 1:

    |d<Z_i>|    <= 2 B + B^2           (||Z_i|| = 1)
    |d<sum Z>|  <= n (2 B + B^2)
    1 - F       <= B^2 / (1 - B)^2     (F = |<psi|psi'>|^2 / ||psi'||^2)

Exact sweeps (CNOT, CZ, X: permutations and sign flips) add no error and
are not counted.
"""

from __future__ import annotations

import math

U32 = 2.0 ** -24
SPLIT = 2.0 ** -16
K = 4.0


def eps_plain(k: int) -> float:
    """Plain FP32 sweep of a gate on k <= 2 targets."""
    L = 2 << k
    return (L + 1) * U32


def eps_fp32_block(k: int, gauss: bool = False) -> float:
    L = 2 << k
    return math.sqrt(2.0) * (L + 3) * U32 if gauss else (L + 1) * U32


def eps_bf16x3_block(k: int) -> float:
    L = 2 << k
    return 3 * SPLIT + (3 * L + 1) * U32


def state_bound(eps_list) -> float:
    """B: bound on ||dpsi||_2 after sweeps with the given eps_g."""
    return K * math.sqrt(sum(2.0 * e * e for e in eps_list))


def z_bound(B: float) -> float:
    return 2.0 * B + B * B


def infidelity_bound(B: float) -> float:
    return B * B / (1.0 - B) ** 2


def plain_circuit_eps(circ) -> list:
    """eps_g of every non-exact gate of a circuit run as plain sweeps."""
    exact = {"x", "y", "z", "swap"}     # entries 0, +-1, +-i (CNOT and CZ are controlled x, z)
    out = []
    for op in circ.ops:
        if op.kind in exact:
            continue
        out.append(eps_plain(len(op.targets)))
    return out


def batch_z_bound(stats: dict, phase_mode: int) -> float:
    """|d<Z_i>| bound for one circuit of a batch plan (``BatchPlan.stats()``):
    at most max_circuit_fused_phases 16 x 16 fused phases (k = 4) in the
    plan's arithmetic plus max_circuit_gate_sweeps FP32 gate sweeps."""
    if phase_mode == 2:
        ef = eps_bf16x3_block(4)
    else:
        ef = eps_fp32_block(4, gauss=True)
    eps = [ef] * int(stats["max_circuit_fused_phases"]) + [eps_plain(2)] * int(stats["max_circuit_gate_sweeps"])
    return z_bound(state_bound(eps))


def plan_z_bound(plan) -> float:
    return batch_z_bound(plan.stats(), plan.info()["config"]["phase_mode"])


def pergate_z_bound(circuits) -> float:
    """The batch run gate by gate (one FP32 sweep per gate)."""
    return z_bound(state_bound([eps_plain(2)] * max(len(c.ops) for c in circuits)))


def sampled_norm_estimate(diff, n: int) -> float:
    """||dpsi||_2 estimated from a uniform sample of amplitude differences:
    sqrt(2^n / S * sum |d_b|^2) (unbiased for ||dpsi||^2)."""
    s = float(sum(abs(complex(d)) ** 2 for d in diff))
    return math.sqrt((2.0 ** n) / max(1, len(diff)) * s)
