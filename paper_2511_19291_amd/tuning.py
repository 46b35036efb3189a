"""Cache of autotuned launch shapes.

The library's autotuners (``sv_batch_autotune`` for the batched launch's tile
shape, ``sv_fused_autotune`` for the fusion width and arithmetic) time
candidates on the device. A choice depends only on the workload's structure
(qubit counts, gate kinds, targets and controls -- not the angles) and the
device, so it is stored in a JSON file under a key of that structure and
reused by later runs.

The cache file is ``$SV_TUNE_CACHE`` if set, else
``~/.cache/sv_mi355x/tune.json``; pass ``path=None`` and ``use_cache=False``
to tune without reading or writing it.
"""

from __future__ import annotations

import hashlib
import json
import os
from typing import Optional, Sequence

from . import sv as svmod


def default_path() -> str:
    return os.environ.get("SV_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "sv_mi355x",
                                                            "tune.json")


def _device_name() -> str:
    import torch

    return torch.cuda.get_device_name(torch.cuda.current_device())


def structure_key(kind: str, circuits: Sequence, extra: str = "", device: Optional[str] = None) -> str:
    """Hash of what the timing depends on: per circuit the qubit count and
    every gate's kind, targets and controls; plus the device name (the
    current GPU's unless given)."""
    h = hashlib.sha1()
    h.update(f"{kind}|{device if device is not None else _device_name()}|{extra}".encode())
    for c in circuits:
        h.update(f"n{c.n}:".encode())
        for op in c.ops:
            h.update(f"{op.kind},{tuple(op.targets)},{tuple(op.controls)};".encode())
    return h.hexdigest()


class TuneCache:
    def __init__(self, path: Optional[str] = None):
        self.path = path or default_path()
        self.data = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, value) -> None:
        self.data[key] = value
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def tuned_batch_config(circuits: Sequence, reps: int = 3, path: Optional[str] = None,
                       use_cache: bool = True) -> dict:
    """The batched launch's configuration for this workload: cached, or
    measured by the library's autotuner and cached."""
    cache = TuneCache(path) if use_cache else None
    key = structure_key("batch", circuits)
    if cache is not None:
        hit = cache.get(key)
        if hit is not None:
            return dict(hit["config"])
    best, trials = svmod.batch_autotune(circuits, reps=reps)
    if cache is not None:
        cache.put(key, {"config": best, "trials": trials})
    return best


def tuned_fusion(state, circuit, modes=(svmod.FUSED_FP32_MFMA, svmod.FUSED_VALU), reps: int = 2,
                 path: Optional[str] = None, use_cache: bool = True) -> dict:
    """Fusion width and mode for this circuit on states of this shape
    (``state`` is overwritten when the autotuner runs)."""
    cache = TuneCache(path) if use_cache else None
    key = structure_key("fusion", [circuit], f"rows{state.batch}|modes{sorted(int(m) for m in modes)}")
    if cache is not None:
        hit = cache.get(key)
        if hit is not None:
            return dict(hit["choice"])
    best, trials = svmod.fused_autotune(state, circuit, modes=modes, reps=reps)
    if cache is not None:
        cache.put(key, {"choice": best, "trials": trials})
    return best
