"""ctypes binding of libsv.so (the C ABI declared in include/sv.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI. PyTorch supplies device memory (a complex64 tensor
of shape [batch, 2^n]) and the stream (the current torch stream), so torch
events and synchronisation see the library's kernels.

Raises ``SvError`` when the library reports a failure and ``RuntimeError``
at import time if libsv.so is missing -- there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SV_LIB_PATH loads another build of the library (the sanitizer test loads a
# build whose host code is instrumented); the default is the in-tree build.
LIB_PATH = os.environ.get("SV_LIB_PATH") or os.path.join(_HERE, "libsv.so")

KINDS = {"h": 1, "x": 2, "y": 3, "z": 4, "s": 5, "sdg": 6, "t": 7, "tdg": 8, "sx": 9,
         "rx": 10, "ry": 11, "rz": 12, "p": 13, "u3": 14, "swap": 15, "rxx": 16, "ryy": 17,
         "rzz": 18, "matrix": 19}

FLAG_ADJOINT = 1
FLAG_CHECK_UNITARY = 2
FUSED_FP32_MFMA = 0
FUSED_BF16X3 = 1
FUSED_VALU = 2
ADJOINT_MFMA = -1          # block_qubits value: the matrix-core blocked backward
BATCH_OUT_STRIDE = 32
MAX_CONTROLS = 3


class SvOp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_targets", C.c_int32), ("targets", C.c_int32 * 2),
                ("n_controls", C.c_int32), ("controls", C.c_int32 * MAX_CONTROLS),
                ("param", C.c_int32 * 3), ("matrix", C.POINTER(C.c_double))]


class SvBlock(C.Structure):
    _fields_ = [("k", C.c_int32), ("targets", C.c_int32 * 6), ("matrix", C.POINTER(C.c_double))]


class SvPauliTerm(C.Structure):
    _fields_ = [("x_mask", C.c_uint64), ("z_mask", C.c_uint64), ("coeff", C.c_double)]


class SvBatchConfig(C.Structure):
    _fields_ = [("tile_bits", C.c_int32), ("threads", C.c_int32), ("reg_min_bits", C.c_int32),
                ("wg_per_cu", C.c_int32), ("phase_mode", C.c_int32), ("fuse_min_gates", C.c_int32),
                ("run_bits", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}

    @classmethod
    def of(cls, d: dict) -> "SvBatchConfig":
        """Fields missing from d take the library's default."""
        base = default_batch_config() if any(f not in d for f, _ in cls._fields_) else {}
        return cls(*[int(d[f] if f in d else base[f]) for f, _ in cls._fields_])


class SvBatchStats(C.Structure):
    _fields_ = [("n_tasks", C.c_int32), ("n_passes", C.c_int32), ("n_phases", C.c_int32),
                ("n_fused_phases", C.c_int32), ("fused_amp_phases", C.c_int64), ("gate_amp_updates", C.c_int64),
                ("max_circuit_fused_phases", C.c_int32), ("max_circuit_gate_sweeps", C.c_int32)]


class SvBatchTrial(C.Structure):
    _fields_ = [("config", SvBatchConfig), ("ms", C.c_double), ("max_dev", C.c_double), ("tol", C.c_double)]


class SvFusionChoice(C.Structure):
    _fields_ = [("max_k", C.c_int32), ("mode", C.c_int32), ("n_sweeps", C.c_int32), ("ms", C.c_double)]

    def as_dict(self) -> dict:
        return {"max_k": int(self.max_k), "mode": int(self.mode), "n_sweeps": int(self.n_sweeps),
                "ms": float(self.ms)}


class SvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsv.so not built ({LIB_PATH}); run paper_2511_19291_amd/csrc/build.py")
    L = C.CDLL(LIB_PATH)
    vp, ip, dp, i64, u64 = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double), C.c_int64, C.c_uint64
    sig = {
        "sv_alloc": [C.c_int, C.c_int, vp, vp, C.POINTER(vp)],
        "sv_free": [vp],
        "sv_device_ptr": [vp, C.POINTER(vp)],
        "sv_state_failed": [vp, ip],
        "sv_inject_hip_error": [vp],
        "sv_reset": [vp, u64],
        "sv_copy_state": [vp, vp, C.c_int],
        "sv_apply_gate": [vp, ip, C.c_int, ip, C.c_int, dp, i64, C.c_uint],
        "sv_run": [vp, C.POINTER(SvOp), C.c_int, dp, i64, C.c_int],
        "sv_apply_fused": [vp, C.POINTER(SvBlock), C.c_int, C.c_int],
        "sv_apply_fused_rows": [vp, C.POINTER(SvBlock), C.c_int, C.c_int],
        "sv_fuse_plan": [C.c_int, C.POINTER(SvOp), C.c_int, dp, C.c_int, C.c_int, C.POINTER(SvBlock),
                         C.c_int, dp, ip],
        "sv_expval_pauli": [vp, C.POINTER(SvPauliTerm), C.c_int, dp],
        "sv_expval_z_all": [vp, dp],
        "sv_expval_z_all_noalloc": [vp, vp],
        "sv_adjoint_grad": [vp, C.POINTER(SvOp), C.c_int, dp, i64, C.c_int, C.POINTER(SvPauliTerm), C.c_int,
                            vp, dp, dp, dp],
        "sv_adjoint_grad_weighted": [vp, C.POINTER(SvOp), C.c_int, dp, i64, C.c_int, C.POINTER(SvPauliTerm),
                                     C.c_int, dp, vp, dp, dp, dp],
        "sv_adjoint_grad_blocked": [vp, C.POINTER(SvOp), C.c_int, dp, i64, C.c_int, C.POINTER(SvPauliTerm),
                                    C.c_int, dp, C.c_int, vp, dp, dp, dp],
        "sv_batch_plan_create": [C.c_int, ip, C.POINTER(C.POINTER(SvOp)), ip, ip, vp, C.POINTER(vp)],
        "sv_batch_default_config": [C.POINTER(SvBatchConfig)],
        "sv_batch_plan_create_ex": [C.c_int, ip, C.POINTER(C.POINTER(SvOp)), ip, ip, C.POINTER(SvBatchConfig), vp,
                                    C.POINTER(vp)],
        "sv_batch_plan_info": [vp, C.POINTER(SvBatchConfig), ip, ip, ip],
        "sv_batch_plan_stats": [vp, C.POINTER(SvBatchStats)],
        "sv_batch_autotune": [C.c_int, ip, C.POINTER(C.POINTER(SvOp)), ip, ip, vp, C.c_int, vp,
                              C.POINTER(SvBatchConfig), C.POINTER(SvBatchTrial), C.c_int, ip],
        "sv_fused_autotune": [vp, C.POINTER(SvOp), C.c_int, dp, C.c_int, C.c_uint32, C.c_int,
                              C.POINTER(SvFusionChoice), C.POINTER(SvFusionChoice), C.c_int, ip],
        "sv_batch_param_layout": [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
        "sv_batch_launch": [vp, vp, vp],
        "sv_batch_launch_pergate": [vp, vp, vp],
        "sv_batch_plan_free": [vp],
        "sv_batch_set_spin_limit": [vp, C.c_int],
        "sv_stream_copy": [vp, vp, u64, vp],
        "sv_sample_exact": [vp, C.c_int, vp, i64, vp],
        "sv_sample_z_estimate": [vp, vp, i64, vp],
        "sv_sample_gaussian": [vp, C.c_int, vp, C.c_double, vp],
        "sv_gaussian_expval_z": [vp, C.c_int, vp, C.c_double, dp],
        "sv_gaussian_expval_z_backward": [vp, C.c_int, vp, C.c_double, dp, vp],
        "sv_adjoint_grad_diag": [vp, C.POINTER(SvOp), C.c_int, dp, i64, C.c_int, vp, C.c_int, vp, dp, dp, dp],
        "sv_adjoint_grad_mfma": [vp, C.POINTER(SvOp), C.c_int, dp, i64, C.c_int, C.POINTER(SvPauliTerm), C.c_int, dp,
                                 vp, dp, dp, dp],
        "sv_check_gate": [C.c_int, ip, C.c_int, ip, C.c_int],
        "sv_sweep_order_tune": [vp, C.POINTER(C.c_float)],
        "sv_sweep_order_set": [vp, u64],
        "sv_sweep_order_get": [vp, C.POINTER(C.c_uint64)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.sv_status_string.argtypes = [C.c_int]
    L.sv_status_string.restype = C.c_char_p
    L.sv_last_error.argtypes = []
    L.sv_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(status: int) -> None:
    if status != 0:
        L = lib()
        raise SvError(status, f"{L.sv_status_string(status).decode()}: {L.sv_last_error().decode()}")


def _iarr(vals: Sequence[int]):
    return (C.c_int * max(1, len(vals)))(*[int(v) for v in vals])


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _cmatrix(m) -> np.ndarray:
    """complex matrix -> interleaved float64 array (kept alive by the caller)."""
    return np.ascontiguousarray(np.asarray(m, dtype=np.complex128)).view(np.float64)


class OpTable:
    """A circuit's gate list as an sv_op array (plus the buffers it points to)."""

    def __init__(self, ops: Iterable, matrices: Optional[dict] = None):
        ops = list(ops)
        self.arr = (SvOp * max(1, len(ops)))()
        self.n = len(ops)
        self._keep: List[np.ndarray] = []
        for i, op in enumerate(ops):
            o = self.arr[i]
            o.kind = KINDS[op.kind]
            o.n_targets = len(op.targets)
            for j, t in enumerate(op.targets):
                o.targets[j] = t
            o.n_controls = len(op.controls)
            for j, c in enumerate(op.controls):
                o.controls[j] = c
            for j in range(3):
                o.param[j] = op.params[j] if j < len(op.params) else -1
            if op.kind == "matrix":
                m = _cmatrix(matrices[i])
                self._keep.append(m)
                o.matrix = _dptr(m)

    @property
    def ptr(self):
        return self.arr


def pauli_terms(terms: Sequence[Tuple[float, int, int]]):
    arr = (SvPauliTerm * max(1, len(terms)))()
    for i, (c, x, z) in enumerate(terms):
        arr[i].x_mask = int(x)
        arr[i].z_mask = int(z)
        arr[i].coeff = float(c)
    return arr


def _params_rows(params, batch: int) -> Tuple[np.ndarray, int, int]:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    if p.ndim == 1:
        return p, 0, int(p.shape[0])
    assert p.ndim == 2 and p.shape[0] == batch, "per-row params must be [batch, n_params]"
    return p, int(p.shape[1]), int(p.shape[1])


class State:
    """A batch of n-qubit complex64 state vectors in GPU memory.

    ``version`` counts the calls that change the amplitudes (reset, copies
    in, gates, fused blocks, the adjoint's un-apply). A caller that keeps a
    result derived from the state -- the autograd layers keep their forward
    output for the backward -- compares it to detect a state that changed
    since. Writes through ``tensor`` by other code are not counted."""

    def __init__(self, n: int, batch: int = 1, device=None, tensor=None):
        import torch

        self.n = n
        self.batch = batch
        if tensor is None:
            tensor = torch.empty((batch, 1 << n), dtype=torch.complex64, device=device or "cuda")
        assert tensor.dtype == torch.complex64 and tensor.is_contiguous() and tensor.numel() == batch << n
        self.tensor = tensor
        self.stream = torch.cuda.current_stream(tensor.device)
        h = C.c_void_p()
        check(lib().sv_alloc(n, batch, C.c_void_p(tensor.data_ptr()), C.c_void_p(self.stream.cuda_stream),
                             C.byref(h)))
        self.h = h
        self.version = 0

    def _changed(self) -> None:
        self.version += 1

    def free(self) -> None:
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.sv_free(h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -- state
    @property
    def failed(self) -> bool:
        """True once a HIP call failed during a call on this state (sticky)."""
        f = C.c_int(0)
        check(lib().sv_state_failed(self.h, C.byref(f)))
        return bool(f.value)

    def reset(self, idx: int = 0) -> "State":
        self._changed()
        check(lib().sv_reset(self.h, idx))
        return self

    def to_numpy(self) -> np.ndarray:
        out = np.empty((self.batch, 1 << self.n), dtype=np.complex64)
        check(lib().sv_copy_state(self.h, out.ctypes.data_as(C.c_void_p), 1))
        return out

    def from_numpy(self, a: np.ndarray) -> "State":
        a = np.ascontiguousarray(np.asarray(a, dtype=np.complex64).reshape(self.batch, 1 << self.n))
        self._changed()
        check(lib().sv_copy_state(self.h, a.ctypes.data_as(C.c_void_p), 0))
        return self

    # -- gates
    def apply_gate(self, matrix, targets: Sequence[int], controls: Sequence[int] = (),
                   adjoint: bool = False, check_unitary: bool = False) -> "State":
        m = np.asarray(matrix, dtype=np.complex128)
        stride = 0
        if m.ndim == 3:
            stride = m.shape[1] * m.shape[2]
        buf = _cmatrix(m)
        flags = (FLAG_ADJOINT if adjoint else 0) | (FLAG_CHECK_UNITARY if check_unitary else 0)
        self._changed()
        check(lib().sv_apply_gate(self.h, _iarr(targets), len(targets), _iarr(controls), len(controls),
                                  _dptr(buf), stride, flags))
        return self

    def run(self, circuit, params=None) -> "State":
        table = OpTable(circuit.ops)
        p, stride, npar = _params_rows(circuit.params if params is None else params, self.batch)
        self._changed()
        check(lib().sv_run(self.h, table.ptr, table.n, _dptr(p) if npar else None, stride, npar))
        return self

    def run_fused(self, circuit, params=None, max_k: int = 5, mode: int = None) -> "State":
        """Apply the circuit with the gates whose angles are equal on every
        row fused into blocks of <= max_k qubits (``fuse_plan``, then
        ``apply_fused`` in ``mode``, FP32 MFMA by default); gates whose
        angles differ between rows (an input encoding) are fused the same
        way with one matrix per row (``apply_fused_rows``) in the
        matrix-core modes from 10 qubits, and run as per-gate sweeps with
        per-row parameters otherwise. The gate order is kept: the circuit is
        cut into maximal runs of row-shared and per-row gates."""
        from .circuits import Circuit

        if mode is None:
            mode = FUSED_FP32_MFMA
        p = np.asarray(circuit.params if params is None else params, dtype=np.float64)
        rows = p.reshape(1, -1) if p.ndim == 1 else p
        same = np.all(rows == rows[:1], axis=0) if rows.shape[1] else np.zeros(0, dtype=bool)
        segs = []
        for op in circuit.ops:
            shared = all(bool(same[j]) for j in op.params)
            if segs and segs[-1][0] == shared:
                segs[-1][1].append(op)
            else:
                segs.append((shared, [op]))
        mfma = mode in (FUSED_FP32_MFMA, FUSED_BF16X3) and circuit.n >= 10
        for shared, ops in segs:
            sub = Circuit(circuit.n, ops, rows[0])
            if shared:
                self.apply_fused(fuse_plan(sub, min(max_k, circuit.n), rows[0]), mode)
            elif mfma and rows.shape[0] == self.batch and len(ops) > 1:
                # the same plan on every row (it depends on the qubits only),
                # each row's matrices from its own angles
                plans = [fuse_plan(sub, min(max_k, 5, circuit.n), rows[r]) for r in range(self.batch)]
                shape = [t for t, _ in plans[0]]
                if any([t for t, _ in pl] != shape for pl in plans):
                    raise RuntimeError("fusion plans differ between rows")
                self.apply_fused_rows([(shape[b], np.stack([pl[b][1] for pl in plans]))
                                       for b in range(len(shape))], mode)
            else:
                self.run(sub, params=p)
        return self

    def run_ops(self, table: "OpTable", start: int, count: int, params: np.ndarray) -> None:
        """Apply ``count`` ops of a prepared table from index ``start``
        (shared parameters)."""
        ptr = C.cast(C.byref(table.arr, start * C.sizeof(SvOp)), C.POINTER(SvOp))
        self._changed()
        check(lib().sv_run(self.h, ptr, count, _dptr(params) if len(params) else None, 0, len(params)))

    def apply_fused(self, blocks: Sequence[Tuple[Sequence[int], np.ndarray]], mode: int = FUSED_FP32_MFMA) -> "State":
        arr = (SvBlock * max(1, len(blocks)))()
        keep = []
        for i, (targets, m) in enumerate(blocks):
            arr[i].k = len(targets)
            for j, t in enumerate(targets):
                arr[i].targets[j] = t
            buf = _cmatrix(m)
            keep.append(buf)
            arr[i].matrix = _dptr(buf)
        self._changed()
        check(lib().sv_apply_fused(self.h, arr, len(blocks), mode))
        return self

    def apply_fused_rows(self, blocks: Sequence[Tuple[Sequence[int], np.ndarray]],
                         mode: int = FUSED_FP32_MFMA) -> "State":
        """Blocks with one matrix per batch row: ``(targets, m)`` with m of
        shape [batch, 2^k, 2^k] (``sv_apply_fused_rows``)."""
        arr = (SvBlock * max(1, len(blocks)))()
        keep = []
        for i, (targets, m) in enumerate(blocks):
            d = 1 << len(targets)
            m = np.asarray(m)
            if m.shape != (self.batch, d, d):
                raise ValueError(f"block {i}: matrices of shape {m.shape}, expected {(self.batch, d, d)}")
            arr[i].k = len(targets)
            for j, t in enumerate(targets):
                arr[i].targets[j] = t
            buf = np.ascontiguousarray(m, dtype=np.complex128).view(np.float64).reshape(-1)
            keep.append(buf)
            arr[i].matrix = _dptr(buf)
        self._changed()
        check(lib().sv_apply_fused_rows(self.h, arr, len(blocks), mode))
        return self

    # -- measurement
    def expval_z_all(self) -> np.ndarray:
        """[batch, n + 1]: <Z_i> for i < n, then ||psi||^2."""
        out = np.zeros((self.batch, self.n + 1), dtype=np.float64)
        check(lib().sv_expval_z_all(self.h, _dptr(out)))
        return out

    def expval_z_all_into(self, out) -> None:
        """Write [batch, n + 1] FP64 <Z_i> and ||psi||^2 into ``out``, a
        caller-allocated contiguous float64 device tensor, with no
        allocation by the library (the fixed-buffer entry point);
        asynchronous on the state's stream."""
        import torch

        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
                and out.is_contiguous() and out.numel() == self.batch * (self.n + 1)):
            raise ValueError(f"out must be a contiguous float64 device tensor of {self.batch * (self.n + 1)} elements")
        check(lib().sv_expval_z_all_noalloc(self.h, C.c_void_p(out.data_ptr())))

    def tune_sweep_order(self) -> np.ndarray:
        """``sv_sweep_order_tune``: time the one-target dense sweep of every
        target >= 7 in both workgroup orders on this state and keep the
        faster per target (for this device and state size). Returns float32
        [n, 2]: median ms in the hardware / XCD-contiguous order (zeros for
        targets that do not use that sweep)."""
        out = np.zeros(2 * self.n, dtype=np.float32)
        check(lib().sv_sweep_order_tune(self.h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out.reshape(self.n, 2)

    def sweep_order(self, xcd_mask: int = None) -> int:
        """Read (and, given ``xcd_mask``, first set) the per-target order
        record of ``sv_sweep_order_set`` / ``sv_sweep_order_get``."""
        if xcd_mask is not None:
            check(lib().sv_sweep_order_set(self.h, C.c_uint64(xcd_mask & (2 ** 64 - 1))))
        out = C.c_uint64(0)
        check(lib().sv_sweep_order_get(self.h, C.byref(out)))
        return int(out.value)

    def expval(self, terms: Sequence[Tuple[float, int, int]]) -> np.ndarray:
        """[batch, n_terms]: coeff_t <P_t>."""
        out = np.zeros((self.batch, len(terms)), dtype=np.float64)
        check(lib().sv_expval_pauli(self.h, pauli_terms(terms), len(terms), _dptr(out)))
        return out

    # -- gradients
    def sample_exact(self, uniforms, row: int = 0):
        """Exact shots (Sec. 4.3.1): one basis index per uniform in [0, 1)
        (a device float64 tensor, or anything torch.as_tensor takes).
        Returns a device int64 tensor; asynchronous on the state's stream."""
        import torch

        u = torch.as_tensor(uniforms, dtype=torch.float64, device=self.tensor.device).contiguous()
        out = torch.empty(u.numel(), dtype=torch.int64, device=self.tensor.device)
        check(lib().sv_sample_exact(self.h, row, C.c_void_p(u.data_ptr()), u.numel(), C.c_void_p(out.data_ptr())))
        self._keep = u          # the kernels read u after this call returns
        return out

    def sample_z_estimate(self, indices):
        """Shot estimates of every <Z_i> from drawn indices (a device int64
        tensor, e.g. from ``sample_exact``): 1 - 2 * (share of the indices
        with bit i set), indices -1 left out. Returns a device float64 tensor
        of length n; asynchronous on the state's stream."""
        import torch

        idx = torch.as_tensor(indices, dtype=torch.int64, device=self.tensor.device).contiguous()
        est = torch.empty(self.n, dtype=torch.float64, device=self.tensor.device)
        check(lib().sv_sample_z_estimate(self.h, C.c_void_p(idx.data_ptr()), idx.numel(), C.c_void_p(est.data_ptr())))
        self._keep_idx = idx    # the kernels read the indices after this call returns
        return est

    def sample_gaussian(self, normals, shots: float, row: int = 0):
        """Gaussian shot histogram (Sec. 4.3.2): y = shots p + sqrt(shots) D S z
        for device float64 normals z of length 2^n. Returns a device float64
        tensor of length 2^n."""
        import torch

        z = torch.as_tensor(normals, dtype=torch.float64, device=self.tensor.device).contiguous()
        assert z.numel() == 1 << self.n
        y = torch.empty(1 << self.n, dtype=torch.float64, device=self.tensor.device)
        check(lib().sv_sample_gaussian(self.h, row, C.c_void_p(z.data_ptr()), float(shots), C.c_void_p(y.data_ptr())))
        self._keep = z
        return y

    def gaussian_expval_z(self, normals, shots: float, row: int = 0) -> np.ndarray:
        """Gaussian shot estimate of every <Z_i> of one row (Sec. 4.3.2),
        from device float64 normals of length 2^n: [n] on the host."""
        import torch

        z = torch.as_tensor(normals, dtype=torch.float64, device=self.tensor.device).contiguous()
        assert z.numel() == 1 << self.n
        est = np.empty(self.n, dtype=np.float64)
        check(lib().sv_gaussian_expval_z(self.h, row, C.c_void_p(z.data_ptr()), float(shots), _dptr(est)))
        return est

    def gaussian_expval_z_backward(self, normals, shots: float, upstream, row: int = 0, out=None):
        """dF/d|psi_b|^2 for F = sum_i upstream[i] E_i (the estimate of
        ``gaussian_expval_z`` with the normals fixed): a device float64
        tensor of length 2^n (written into ``out`` when given)."""
        import torch

        z = torch.as_tensor(normals, dtype=torch.float64, device=self.tensor.device).contiguous()
        assert z.numel() == 1 << self.n
        g = np.ascontiguousarray(np.asarray(upstream, dtype=np.float64).reshape(self.n))
        w = out if out is not None else torch.empty(1 << self.n, dtype=torch.float64, device=self.tensor.device)
        assert w.dtype == torch.float64 and w.is_contiguous() and w.numel() == 1 << self.n
        check(lib().sv_gaussian_expval_z_backward(self.h, row, C.c_void_p(z.data_ptr()), float(shots), _dptr(g),
                                                  C.c_void_p(w.data_ptr())))
        self._keep = z
        return w

    def adjoint_grad_diag(self, circuit, weights, params=None, block_qubits: int = 0,
                          lambda_tensor=None) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """Adjoint gradient for the diagonal observable diag(weights), a
        device float64 tensor [batch, 2^n]; returns (loss, grad, drift) as
        ``adjoint_grad``."""
        table = OpTable(circuit.ops)
        p, stride, npar = _params_rows(circuit.params if params is None else params, self.batch)
        assert weights.is_contiguous() and weights.numel() == self.batch << self.n
        grad = np.zeros((self.batch, max(npar, 1)), dtype=np.float64)
        loss = np.zeros(self.batch, dtype=np.float64)
        drift = np.zeros(self.batch, dtype=np.float64)
        lam = C.c_void_p(lambda_tensor.data_ptr()) if lambda_tensor is not None else None
        self._changed()
        check(lib().sv_adjoint_grad_diag(self.h, table.ptr, table.n, _dptr(p) if npar else None, stride, npar,
                                         C.c_void_p(weights.data_ptr()), block_qubits, lam, _dptr(grad), _dptr(loss),
                                         _dptr(drift)))
        return loss, grad[:, :npar], drift

    def adjoint_grad(self, circuit, terms: Sequence[Tuple[float, int, int]], params=None,
                     lambda_tensor=None, coeff_rows=None, block_qubits: int = 0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """The state must hold the forward output of ``circuit``. Returns
        (loss [batch], grad [batch, n_params], drift [batch]) and leaves the
        recomputed start state in the state. ``coeff_rows`` ([batch, n_terms])
        replaces the terms' coefficients row by row. ``block_qubits`` 3, 4 or
        5 runs the blocked backward (one sweep per block of gates),
        ``ADJOINT_MFMA`` the blocked backward on the matrix cores, 0 the
        per-gate one."""
        table = OpTable(circuit.ops)
        p, stride, npar = _params_rows(circuit.params if params is None else params, self.batch)
        grad = np.zeros((self.batch, max(npar, 1)), dtype=np.float64)
        loss = np.zeros(self.batch, dtype=np.float64)
        drift = np.zeros(self.batch, dtype=np.float64)
        lam = C.c_void_p(lambda_tensor.data_ptr()) if lambda_tensor is not None else None
        pp = _dptr(p) if npar else None
        self._changed()
        if block_qubits == ADJOINT_MFMA:
            cr = None
            if coeff_rows is not None:
                cr = np.ascontiguousarray(np.asarray(coeff_rows, dtype=np.float64).reshape(self.batch, len(terms)))
            check(lib().sv_adjoint_grad_mfma(self.h, table.ptr, table.n, pp, stride, npar, pauli_terms(terms),
                                             len(terms), _dptr(cr) if cr is not None else None, lam, _dptr(grad),
                                             _dptr(loss), _dptr(drift)))
        elif block_qubits:
            cr = None
            if coeff_rows is not None:
                cr = np.ascontiguousarray(np.asarray(coeff_rows, dtype=np.float64).reshape(self.batch, len(terms)))
            check(lib().sv_adjoint_grad_blocked(self.h, table.ptr, table.n, pp, stride, npar, pauli_terms(terms),
                                                len(terms), _dptr(cr) if cr is not None else None, block_qubits, lam,
                                                _dptr(grad), _dptr(loss), _dptr(drift)))
        elif coeff_rows is None:
            check(lib().sv_adjoint_grad(self.h, table.ptr, table.n, pp, stride, npar, pauli_terms(terms), len(terms),
                                        lam, _dptr(grad), _dptr(loss), _dptr(drift)))
        else:
            cr = np.ascontiguousarray(np.asarray(coeff_rows, dtype=np.float64).reshape(self.batch, len(terms)))
            check(lib().sv_adjoint_grad_weighted(self.h, table.ptr, table.n, pp, stride, npar, pauli_terms(terms),
                                                 len(terms), _dptr(cr), lam, _dptr(grad), _dptr(loss), _dptr(drift)))
        return loss, grad[:, :npar], drift


def fuse_plan(circuit, max_k: int = 5, params=None) -> List[Tuple[Tuple[int, ...], np.ndarray]]:
    """Host-only fusion planner: blocks (targets, complex128 matrix)."""
    table = OpTable(circuit.ops)
    p = np.ascontiguousarray(np.asarray(circuit.params if params is None else params, dtype=np.float64))
    max_blocks = max(1, len(circuit.ops))
    blocks = (SvBlock * max_blocks)()
    mats = np.zeros(max_blocks * (4 ** max_k) * 2, dtype=np.float64)
    nb = C.c_int()
    check(lib().sv_fuse_plan(circuit.n, table.ptr, table.n, _dptr(p) if len(p) else None, len(p), max_k,
                             blocks, max_blocks, _dptr(mats), C.byref(nb)))
    base = mats.ctypes.data
    out = []
    for i in range(nb.value):
        b = blocks[i]
        d = 1 << b.k
        off = (C.cast(b.matrix, C.c_void_p).value - base) // 8
        m = mats[off: off + 2 * d * d].view(np.complex128).reshape(d, d).copy()
        out.append((tuple(b.targets[j] for j in range(b.k)), m))
    return out


def _batch_arrays(circuits, tables):
    nc = len(circuits)
    nq = _iarr([c.n for c in circuits])
    nops = _iarr([t.n for t in tables])
    npar = _iarr([c.n_params for c in circuits])
    ops_arr = (C.POINTER(SvOp) * nc)(*[C.cast(t.arr, C.POINTER(SvOp)) for t in tables])
    return nc, nq, ops_arr, nops, npar


def default_batch_config() -> dict:
    c = SvBatchConfig()
    check(lib().sv_batch_default_config(C.byref(c)))
    return c.as_dict()


class BatchPlan:
    """Many independent circuits (uneven qubit counts) run by one persistent
    kernel launch captured in a hipGraph; every circuit starts from |0..0>
    and yields all <Z_i>. ``config`` (a dict with the fields of
    ``sv_batch_config``) sets the launch shape; None takes the default."""

    def __init__(self, circuits: Sequence, device=None, config: Optional[dict] = None):
        import torch

        self.circuits = list(circuits)
        self.stream = torch.cuda.current_stream(device)
        self.tables = [OpTable(c.ops) for c in self.circuits]
        nc, nq, ops_arr, nops, npar = _batch_arrays(self.circuits, self.tables)
        h = C.c_void_p()
        cfg = C.byref(SvBatchConfig.of(config)) if config is not None else None
        check(lib().sv_batch_plan_create_ex(nc, nq, ops_arr, nops, npar, cfg, C.c_void_p(self.stream.cuda_stream),
                                            C.byref(h)))
        self.h = h
        offs = (C.c_int64 * nc)()
        total = C.c_int64()
        check(lib().sv_batch_param_layout(self.h, offs, C.byref(total)))
        self.offsets = [int(x) for x in offs]
        self.total = int(total.value)

    def info(self) -> dict:
        """Effective configuration, persistent grid, tile tasks and passes."""
        cfg = SvBatchConfig()
        grid, tasks, passes = C.c_int(), C.c_int(), C.c_int()
        check(lib().sv_batch_plan_info(self.h, C.byref(cfg), C.byref(grid), C.byref(tasks), C.byref(passes)))
        return {"config": cfg.as_dict(), "grid": grid.value, "n_tasks": tasks.value, "n_passes": passes.value}

    def stats(self) -> dict:
        """Work counts of the plan (sv_batch_plan_stats)."""
        st = SvBatchStats()
        check(lib().sv_batch_plan_stats(self.h, C.byref(st)))
        return {f: int(getattr(st, f)) for f, _ in st._fields_}

    def pack(self, params_list=None):
        """Device FP64 parameter block in the plan's layout."""
        import torch

        flat = np.zeros(max(self.total, 1), dtype=np.float64)
        for i, (c, off) in enumerate(zip(self.circuits, self.offsets)):
            p = c.params if params_list is None else params_list[i]
            flat[off: off + c.n_params] = p
        return torch.from_numpy(flat).to(device=self.stream.device)

    def out_buffer(self):
        import torch

        return torch.zeros((len(self.circuits), BATCH_OUT_STRIDE), dtype=torch.float64, device=self.stream.device)

    def set_spin_limit(self, limit: int) -> None:
        """Testing hook of the inter-pass wait (``sv_batch_set_spin_limit``):
        polls before a wait gives up and the circuit's outputs become NaN;
        negative: give up at once. 2**24 is the default."""
        check(lib().sv_batch_set_spin_limit(self.h, int(limit)))

    def launch(self, dev_params, dev_out, pergate: bool = False) -> None:
        f = lib().sv_batch_launch_pergate if pergate else lib().sv_batch_launch
        check(f(self.h, C.c_void_p(dev_params.data_ptr()), C.c_void_p(dev_out.data_ptr())))

    def run(self, params_list=None, pergate: bool = False) -> np.ndarray:
        dp = self.pack(params_list)
        out = self.out_buffer()
        self.launch(dp, out, pergate)
        self.stream.synchronize()
        return out.cpu().numpy()

    def free(self) -> None:
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.sv_batch_plan_free(h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def batch_autotune(circuits: Sequence, reps: int = 3, device=None, params_list=None):
    """Time the batch under the library's staged search over launch shapes.
    Returns (best config dict, list of trials {config, ms, max_dev, tol})."""
    import torch

    circuits = list(circuits)
    stream = torch.cuda.current_stream(device)
    tables = [OpTable(c.ops) for c in circuits]
    nc, nq, ops_arr, nops, npar = _batch_arrays(circuits, tables)
    total = sum(c.n_params for c in circuits)
    flat = np.zeros(max(total, 1), dtype=np.float64)
    off = 0
    for i, c in enumerate(circuits):      # the layout is the circuits' parameter rows in order
        flat[off: off + c.n_params] = c.params if params_list is None else params_list[i]
        off += c.n_params
    dparams = torch.from_numpy(flat).to(device=stream.device)
    best = SvBatchConfig()
    cap = 64
    trials = (SvBatchTrial * cap)()
    nt = C.c_int()
    check(lib().sv_batch_autotune(nc, nq, ops_arr, nops, npar, C.c_void_p(dparams.data_ptr()), reps,
                                  C.c_void_p(stream.cuda_stream), C.byref(best), trials, cap, C.byref(nt)))
    out = [{"config": trials[i].config.as_dict(), "ms": float(trials[i].ms), "max_dev": float(trials[i].max_dev),
            "tol": float(trials[i].tol)} for i in range(min(nt.value, cap))]
    return best.as_dict(), out


def fused_autotune(state: "State", circuit, modes: Sequence[int] = (FUSED_FP32_MFMA, FUSED_VALU), reps: int = 2,
                   params=None):
    """Time the circuit on ``state`` as plain sweeps and as fused blocks of
    each width in the allowed modes (the state is overwritten). Returns (best
    choice dict, list of trial dicts); mode -1 means plain per-gate sweeps."""
    table = OpTable(circuit.ops)
    p = np.ascontiguousarray(np.asarray(circuit.params if params is None else params, dtype=np.float64))
    mask = 0
    for m in modes:
        mask |= 1 << int(m)
    best = SvFusionChoice()
    cap = 16
    trials = (SvFusionChoice * cap)()
    nt = C.c_int()
    check(lib().sv_fused_autotune(state.h, table.ptr, table.n, _dptr(p) if len(p) else None, len(p), mask, reps,
                                  C.byref(best), trials, cap, C.byref(nt)))
    return best.as_dict(), [trials[i].as_dict() for i in range(min(nt.value, cap))]
