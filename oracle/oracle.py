"""Python driver of the C oracle -- TEST INFRASTRUCTURE.

Plain complex128 simulation of a circuit, Pauli expectation values and three
exact-gradient routes (parameter shift, central finite differences and the
recompute-by-inverse adjoint of Sec. 4.4). The heavy loops live in
sv_oracle.c; this module only sequences them.

Circuits are duck-typed: any object with ``n``, ``ops`` (each with ``kind``,
``targets``, ``controls``, ``params``) and ``params`` works. Pauli terms are
(coeff, x_mask, z_mask) with bit q of x_mask set for X or Y on qubit q and bit
q of z_mask set for Z or Y.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Sequence, Tuple

import numpy as np

from . import build as _build

_LIB = None
MAX_K = 6

Term = Tuple[float, int, int]


def load() -> C.CDLL:
    """Load liboracle.so, building it first if it is missing. The
    environment variable SV_ORACLE_LIB names another build of sv_oracle.c to
    load instead (the sanitizer test runs the pins on an instrumented one)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    other = os.environ.get("SV_ORACLE_LIB")
    if other:
        _LIB = bind(C.CDLL(other))
        return _LIB
    if not os.path.exists(_build.LIB):
        _build.build()
    _LIB = bind(C.CDLL(_build.LIB))
    return _LIB


def bind(lib: C.CDLL) -> C.CDLL:
    """Declare the C signatures on a loaded oracle library."""
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    lib.orc_gate_matrix.argtypes = [C.c_char_p, dp, dp]
    lib.orc_gate_matrix.restype = C.c_int
    lib.orc_gate_dmatrix.argtypes = [C.c_char_p, dp, C.c_int, dp]
    lib.orc_gate_dmatrix.restype = C.c_int
    lib.orc_apply.argtypes = [dp, C.c_int, C.c_int, ip, C.c_int, ip, dp]
    lib.orc_apply.restype = C.c_int
    lib.orc_project_controls.argtypes = [dp, C.c_int, C.c_int, ip]
    lib.orc_project_controls.restype = None
    lib.orc_basis.argtypes = [dp, C.c_int, C.c_uint64]
    lib.orc_basis.restype = None
    lib.orc_expval_pauli.argtypes = [dp, C.c_int, C.c_uint64, C.c_uint64, dp, dp]
    lib.orc_expval_pauli.restype = None
    lib.orc_expval_z_all.argtypes = [dp, C.c_int, dp]
    lib.orc_expval_z_all.restype = None
    lib.orc_inner.argtypes = [dp, dp, C.c_int, dp, dp]
    lib.orc_inner.restype = None
    u64p = C.POINTER(C.c_uint64)
    lib.orc_apply_pauli_sum.argtypes = [dp, C.c_int, C.c_int, u64p, u64p, dp, dp]
    lib.orc_apply_pauli_sum.restype = None
    lib.orc_prob_cdf.argtypes = [dp, C.c_int, dp]
    lib.orc_prob_cdf.restype = None
    i64p = C.POINTER(C.c_int64)
    lib.orc_sample_exact.argtypes = [dp, C.c_int, dp, C.c_int64, i64p]
    lib.orc_sample_exact.restype = None
    lib.orc_sample_gaussian.argtypes = [dp, C.c_int, dp, C.c_double, dp]
    lib.orc_sample_gaussian.restype = None
    lib.orc_gaussian_z.argtypes = [dp, C.c_int, dp, C.c_double, dp, dp]
    lib.orc_gaussian_z.restype = None
    lib.orc_gaussian_z_weights.argtypes = [dp, C.c_int, dp, C.c_double, dp, dp]
    lib.orc_gaussian_z_weights.restype = None
    return lib


class using_library:
    """Context manager: run the oracle functions on another build of
    sv_oracle.c (the mutation tests plant mistakes in a copy)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _LIB
        self.saved = load()
        _LIB = bind(C.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _LIB
        _LIB = self.saved
        return False


def _dptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iarr(vals: Sequence[int]):
    arr = (C.c_int * max(1, len(vals)))(*vals)
    return arr


# ------------------------------------------------------------------ state

def basis_state(n: int, idx: int = 0) -> np.ndarray:
    """e_idx in C^(2^n), complex128."""
    psi = np.empty(1 << n, dtype=np.complex128)
    load().orc_basis(_dptr(psi.view(np.float64)), n, idx)
    return psi


def gate_matrix(kind: str, prm: Sequence[float] = ()) -> np.ndarray:
    """The 2^k x 2^k complex128 matrix of a gate kind (first target = most
    significant index bit)."""
    p = np.zeros(4, dtype=np.float64)
    p[: len(prm)] = prm
    m = np.zeros((1 << MAX_K) ** 2, dtype=np.complex128)
    k = load().orc_gate_matrix(kind.encode(), _dptr(p), _dptr(m.view(np.float64)))
    if k < 0:
        raise ValueError(f"oracle: unknown gate kind {kind!r}")
    d = 1 << k
    return m[: d * d].reshape(d, d).copy()


def gate_dmatrix(kind: str, prm: Sequence[float], j: int) -> np.ndarray:
    """d/d prm[j] of the gate matrix."""
    p = np.zeros(4, dtype=np.float64)
    p[: len(prm)] = prm
    m = np.zeros((1 << MAX_K) ** 2, dtype=np.complex128)
    k = load().orc_gate_dmatrix(kind.encode(), _dptr(p), j, _dptr(m.view(np.float64)))
    if k < 0:
        raise ValueError(f"oracle: kind {kind!r} has no parameter {j}")
    d = 1 << k
    return m[: d * d].reshape(d, d).copy()


def apply_matrix(psi: np.ndarray, n: int, m: np.ndarray, targets: Sequence[int],
                 controls: Sequence[int] = ()) -> None:
    """In place: psi <- (M on targets, controlled by controls) psi."""
    m = np.ascontiguousarray(m, dtype=np.complex128)
    k = len(targets)
    assert m.shape == (1 << k, 1 << k)
    rc = load().orc_apply(_dptr(psi.view(np.float64)), n, k, _iarr(targets), len(controls),
                          _iarr(controls), _dptr(m.view(np.float64)))
    if rc != 0:
        raise ValueError(f"oracle: bad gate targets={targets} controls={controls} n={n}")


def _op_values(op, params: np.ndarray) -> List[float]:
    return [float(params[i]) for i in op.params]


def apply_op(psi: np.ndarray, n: int, op, params: np.ndarray, dagger: bool = False) -> None:
    m = gate_matrix(op.kind, _op_values(op, params))
    if dagger:
        m = m.conj().T.copy()
    apply_matrix(psi, n, m, op.targets, op.controls)


def run(circuit, params: np.ndarray | None = None, psi: np.ndarray | None = None) -> np.ndarray:
    """Final state of the circuit from |0..0> (or from ``psi``, in place)."""
    params = circuit.params if params is None else params
    if psi is None:
        psi = basis_state(circuit.n, 0)
    for op in circuit.ops:
        apply_op(psi, circuit.n, op, params)
    return psi


def run_inverse(circuit, psi: np.ndarray, params: np.ndarray | None = None) -> np.ndarray:
    """Un-apply the circuit: gates in reverse order, each as M^* (Sec. 4.4)."""
    params = circuit.params if params is None else params
    for op in reversed(circuit.ops):
        apply_op(psi, circuit.n, op, params, dagger=True)
    return psi


# ------------------------------------------------------------ expectation

def expval_pauli(psi: np.ndarray, n: int, x_mask: int, z_mask: int) -> Tuple[float, float]:
    re = C.c_double()
    im = C.c_double()
    load().orc_expval_pauli(_dptr(psi.view(np.float64)), n, x_mask, z_mask, C.byref(re), C.byref(im))
    return re.value, im.value


def expval_z_all(psi: np.ndarray, n: int) -> Tuple[np.ndarray, float]:
    """(<Z_0>, ..., <Z_{n-1}>) and ||psi||^2."""
    out = np.zeros(n + 1, dtype=np.float64)
    load().orc_expval_z_all(_dptr(psi.view(np.float64)), n, _dptr(out))
    return out[:n].copy(), float(out[n])


def expval_terms(psi: np.ndarray, n: int, terms: Iterable[Term]) -> float:
    """sum_t coeff_t <P_t>."""
    return float(sum(c * expval_pauli(psi, n, x, z)[0] for c, x, z in terms))


def inner(a: np.ndarray, b: np.ndarray, n: int) -> complex:
    re = C.c_double()
    im = C.c_double()
    load().orc_inner(_dptr(a.view(np.float64)), _dptr(b.view(np.float64)), n, C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def apply_pauli_sum(psi: np.ndarray, n: int, terms: Sequence[Term]) -> np.ndarray:
    """O psi for O = sum_t coeff_t P_t (a new array)."""
    out = np.empty_like(psi)
    nt = len(terms)
    xm = (C.c_uint64 * nt)(*[int(t[1]) for t in terms])
    zm = (C.c_uint64 * nt)(*[int(t[2]) for t in terms])
    cf = np.asarray([float(t[0]) for t in terms], dtype=np.float64)
    load().orc_apply_pauli_sum(_dptr(psi.view(np.float64)), n, nt, xm, zm, _dptr(cf),
                               _dptr(out.view(np.float64)))
    return out


def loss(circuit, terms: Sequence[Term], params: np.ndarray | None = None) -> float:
    """L(params) = <psi(params)| O |psi(params)> from |0..0>."""
    return expval_terms(run(circuit, params), circuit.n, terms)


# -------------------------------------------------------------- gradients

# Kinds for which the two-term shift rule with shift pi/2 is exact as a
# function of one parameter (generator with two eigenvalues 1/2 apart).
_SHIFT_OK_UNCONTROLLED = ("rx", "ry", "rz", "rxx", "ryy", "rzz", "p", "u3")
_SHIFT_OK_CONTROLLED = ("p",)


def grad_param_shift(circuit, terms: Sequence[Term], params: np.ndarray | None = None) -> np.ndarray:
    """Exact gradient by the parameter-shift rule
    dL/dtheta = [L(theta + pi/2) - L(theta - pi/2)] / 2, applied to each gate
    occurrence of each parameter (parameters shared by several gates sum)."""
    params = np.array(circuit.params if params is None else params, dtype=np.float64)
    # give every (gate, slot) occurrence its own parameter so it can shift alone
    occ = []
    for gi, op in enumerate(circuit.ops):
        for j, p in enumerate(op.params):
            ok = _SHIFT_OK_CONTROLLED if op.controls else _SHIFT_OK_UNCONTROLLED
            if op.kind not in ok:
                raise ValueError(f"parameter shift not exact for {'c' * len(op.controls)}{op.kind}")
            occ.append((gi, j, p))
    grad = np.zeros(len(params), dtype=np.float64)
    for gi, j, p in occ:
        vals = []
        for sgn in (+1.0, -1.0):
            psi = basis_state(circuit.n, 0)
            for gk, op in enumerate(circuit.ops):
                v = _op_values(op, params)
                if gk == gi:
                    v[j] += sgn * np.pi / 2
                apply_matrix(psi, circuit.n, gate_matrix(op.kind, v), op.targets, op.controls)
            vals.append(expval_terms(psi, circuit.n, terms))
        grad[p] += 0.5 * (vals[0] - vals[1])
    return grad


def grad_finite_diff(circuit, terms: Sequence[Term], h: float = 1e-4,
                     params: np.ndarray | None = None, which: Sequence[int] | None = None) -> np.ndarray:
    """Central finite differences [L(p + h e_i) - L(p - h e_i)] / (2h)."""
    params = np.array(circuit.params if params is None else params, dtype=np.float64)
    which = range(len(params)) if which is None else which
    grad = np.zeros(len(params), dtype=np.float64)
    for i in which:
        pp = params.copy()
        pp[i] += h
        pm = params.copy()
        pm[i] -= h
        grad[i] = (loss(circuit, terms, pp) - loss(circuit, terms, pm)) / (2 * h)
    return grad


def grad_adjoint(circuit, terms: Sequence[Term], params: np.ndarray | None = None,
                 psi_final: np.ndarray | None = None) -> Tuple[float, np.ndarray, float]:
    """Adjoint-method gradient by un-applying gates (Sec. 4.4: the layer input
    is recomputed as x = U^* y instead of stored).

    With psi_l = U_l psi_{l-1} and L = <psi_L|O|psi_L>:
        lam <- O psi_L
        for l = L..1:
            psi <- U_l^* psi                         (now psi_{l-1})
            g[p] += 2 Re <lam | dU_l/dtheta_p | psi> (each parameter of U_l)
            lam <- U_l^* lam
    Returns (L, grad, ||psi_0_recomputed - e_0||).
    """
    params = np.asarray(circuit.params if params is None else params, dtype=np.float64)
    n = circuit.n
    psi = run(circuit, params) if psi_final is None else psi_final.copy()
    lam = apply_pauli_sum(psi, n, terms)
    L = inner(psi, lam, n).real
    grad = np.zeros(len(params), dtype=np.float64)
    for op in reversed(circuit.ops):
        v = _op_values(op, params)
        m = gate_matrix(op.kind, v)
        apply_matrix(psi, n, m.conj().T.copy(), op.targets, op.controls)
        for j, p in enumerate(op.params):
            dm = gate_dmatrix(op.kind, v, j)
            mu = psi.copy()
            if op.controls:
                load().orc_project_controls(_dptr(mu.view(np.float64)), n, len(op.controls),
                                            _iarr(op.controls))
                # on the controlled subspace the gate is M, elsewhere identity:
                # the derivative is dM there and 0 elsewhere
            apply_matrix(mu, n, dm, op.targets, op.controls)
            grad[p] += 2.0 * inner(lam, mu, n).real
        apply_matrix(lam, n, m.conj().T.copy(), op.targets, op.controls)
    e0 = basis_state(n, 0)
    drift = float(np.linalg.norm(psi - e0))
    return L, grad, drift


# ------------------------------------------------------------------ shots

def prob_cdf(psi: np.ndarray, n: int) -> np.ndarray:
    """cdf[b] = sum_{c <= b} |psi_c|^2 (compensated running sum)."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty(1 << n, dtype=np.float64)
    load().orc_prob_cdf(_dptr(psi.view(np.float64)), n, _dptr(out))
    return out


def sample_exact(psi: np.ndarray, n: int, uniforms: np.ndarray) -> np.ndarray:
    """Exact shots (Sec. 4.3.1): for each u the smallest b with
    cdf[b] > u T (clamped below T); -1 for a zero state."""
    cdf = prob_cdf(psi, n)
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    out = np.empty(len(u), dtype=np.int64)
    load().orc_sample_exact(_dptr(cdf), n, _dptr(u), len(u), out.ctypes.data_as(C.POINTER(C.c_int64)))
    return out


def sample_gaussian(psi: np.ndarray, n: int, normals: np.ndarray, shots: float) -> np.ndarray:
    """Gaussian shot histogram (Sec. 4.3.2): y = shots p + sqrt(shots) D S z
    with the Householder reflection S (z's last entry is taken as 0)."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    z = np.ascontiguousarray(normals, dtype=np.float64)
    assert len(z) == 1 << n
    y = np.empty(1 << n, dtype=np.float64)
    load().orc_sample_gaussian(_dptr(psi.view(np.float64)), n, _dptr(z), float(shots), _dptr(y))
    return y


def gaussian_z(psi: np.ndarray, n: int, normals: np.ndarray, shots: float) -> np.ndarray:
    """Gaussian shot estimate of every <Z_i> (Sec. 4.3.2): E_i = (1/shots)
    sum_b y_b s_i(b), y the histogram of ``sample_gaussian``."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    z = np.ascontiguousarray(normals, dtype=np.float64)
    assert len(z) == 1 << n
    est = np.empty(n, dtype=np.float64)
    work = np.empty(1 << n, dtype=np.float64)
    load().orc_gaussian_z(_dptr(psi.view(np.float64)), n, _dptr(z), float(shots), _dptr(est), _dptr(work))
    return est


def gaussian_z_weights(psi: np.ndarray, n: int, normals: np.ndarray, shots: float, upstream) -> np.ndarray:
    """dF/d|psi_b|^2 for F = sum_i upstream_i E_i (E from ``gaussian_z``,
    the normals held fixed): the diagonal observable whose adjoint gives
    dF/dtheta."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    z = np.ascontiguousarray(normals, dtype=np.float64)
    g = np.ascontiguousarray(upstream, dtype=np.float64)
    assert len(z) == 1 << n and len(g) == n
    w = np.empty(1 << n, dtype=np.float64)
    load().orc_gaussian_z_weights(_dptr(psi.view(np.float64)), n, _dptr(z), float(shots), _dptr(g), _dptr(w))
    return w
