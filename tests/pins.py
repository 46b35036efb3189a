"""Independent constructions used to pin the oracle (test side only).

Nothing here calls the oracle's arithmetic. Two other routes to the same
results:

* ``alg1_apply``: the paper's Alg. 1 taken literally with numpy -- view the
  state as a rank-n tensor, move the gate's qubit axes to the front
  (MoveDim), contract with M (mm), move the axes back (MoveDim^-1).
* ``embed_kron``: the full 2^n x 2^n operator of a gate as a sum of Kronecker
  products of matrix units, with control projectors: U = I - Pi_C + Pi_C U_M.

Gate matrices come from scipy's matrix exponential of Pauli generators and
from hand-written closed forms, not from the oracle.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI = {"I": I2, "X": PX, "Y": PY, "Z": PZ}


def expm_rotation(pauli: np.ndarray, theta: float) -> np.ndarray:
    """exp(-i theta P / 2) by scipy's matrix exponential."""
    return sla.expm(-0.5j * theta * pauli)


def textbook_matrix(kind: str, prm=()) -> np.ndarray:
    """Gate matrices from definitions independent of the oracle's code:
    rotations by matrix exponential, u3 as a product of rotations times the
    global phase e^{i(phi+lambda)/2}."""
    if kind in ("rx", "ry", "rz"):
        return expm_rotation({"rx": PX, "ry": PY, "rz": PZ}[kind], prm[0])
    if kind in ("rxx", "ryy", "rzz"):
        p = {"rxx": PX, "ryy": PY, "rzz": PZ}[kind]
        return expm_rotation(np.kron(p, p), prm[0])
    if kind == "p":
        return np.exp(0.5j * prm[0]) * expm_rotation(PZ, prm[0])
    if kind == "u3":
        t, f, lam = prm
        return np.exp(0.5j * (f + lam)) * (expm_rotation(PZ, f) @ expm_rotation(PY, t) @ expm_rotation(PZ, lam))
    if kind == "h":
        return (PX + PZ) / np.sqrt(2)
    if kind == "x":
        return PX.copy()
    if kind == "y":
        return PY.copy()
    if kind == "z":
        return PZ.copy()
    if kind == "s":
        return sla.sqrtm(PZ)
    if kind == "sdg":
        return sla.sqrtm(PZ).conj().T
    if kind == "t":
        return sla.sqrtm(sla.sqrtm(PZ))
    if kind == "tdg":
        return sla.sqrtm(sla.sqrtm(PZ)).conj().T
    if kind == "sx":
        return sla.sqrtm(PX)
    if kind == "swap":
        m = np.zeros((4, 4), dtype=np.complex128)
        for a in range(2):
            for b in range(2):
                m[(b << 1) | a, (a << 1) | b] = 1
        return m
    raise ValueError(kind)


def alg1_apply(psi: np.ndarray, n: int, m: np.ndarray, targets, controls=()) -> np.ndarray:
    """Alg. 1 with numpy: MoveDim, mm, MoveDim^-1 on the rank-n tensor view.

    C-order reshape puts the most significant index bit first, so qubit q
    (bit q) is tensor axis n-1-q. Controls restrict the update to the slice
    where every control axis is 1."""
    k = len(targets)
    x = psi.reshape((2,) * n).copy()
    out = x.copy()
    sl = [slice(None)] * n
    for c in controls:
        sl[n - 1 - c] = 1
    sub = x[tuple(sl)]
    # axes of the sub-tensor: the control axes are gone; renumber the rest
    keep = [ax for ax in range(n) if ax not in {n - 1 - c for c in controls}]
    axes = [keep.index(n - 1 - t) for t in targets]
    moved = np.moveaxis(sub, axes, list(range(k)))            # MoveDim
    shp = moved.shape
    prod = (m @ moved.reshape(1 << k, -1)).reshape(shp)       # mm(M, X)
    back = np.moveaxis(prod, list(range(k)), axes)            # MoveDim^-1
    out[tuple(sl)] = back
    return out.reshape(-1)


def _unit(r: int, s: int) -> np.ndarray:
    e = np.zeros((2, 2), dtype=np.complex128)
    e[r, s] = 1
    return e


def kron_chain(factors_by_qubit: dict, n: int) -> np.ndarray:
    """Kronecker product with qubit n-1 leftmost (qubit q = bit q)."""
    out = np.ones((1, 1), dtype=np.complex128)
    for q in reversed(range(n)):
        out = np.kron(out, factors_by_qubit.get(q, I2))
    return out


def embed_kron(m: np.ndarray, n: int, targets, controls=()) -> np.ndarray:
    """Full operator: U_M = sum_{r,s} M[r,s] kron_q F_q with F at target j the
    matrix unit |r_j><s_j| (r_j = bit k-1-j of r), identity elsewhere; then
    U = I - Pi_C + Pi_C U_M with Pi_C the projector onto control bits = 1."""
    k = len(targets)
    d = 1 << k
    um = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for r in range(d):
        for s in range(d):
            if m[r, s] == 0:
                continue
            f = {t: _unit((r >> (k - 1 - j)) & 1, (s >> (k - 1 - j)) & 1) for j, t in enumerate(targets)}
            um += m[r, s] * kron_chain(f, n)
    if not controls:
        return um
    pc = kron_chain({c: _unit(1, 1) for c in controls}, n)
    return np.eye(1 << n, dtype=np.complex128) - pc + pc @ um


def pauli_matrix(n: int, x_mask: int, z_mask: int) -> np.ndarray:
    f = {}
    for q in range(n):
        xb, zb = (x_mask >> q) & 1, (z_mask >> q) & 1
        f[q] = {(0, 0): I2, (1, 0): PX, (1, 1): PY, (0, 1): PZ}[(xb, zb)]
    return kron_chain(f, n)


def random_state(n: int, rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary: QR of a complex Gaussian with the phase fix."""
    z = (rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph
