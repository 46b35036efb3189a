"""Host-side logic of the autotuning cache (no GPU): structure keys ignore
the angles but see every structural change; the JSON store round-trips."""

import json

import numpy as np

from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import tuning


def test_key_ignores_angles_and_sees_structure():
    a = C.encoded_ansatz(10, 2, np.random.default_rng(1))
    b = C.encoded_ansatz(10, 2, np.random.default_rng(2))        # same structure, other angles
    assert not np.allclose(a.params, b.params)
    k = lambda cs, **kw: tuning.structure_key("batch", cs, device="dev0", **kw)
    assert k([a]) == k([b])
    assert k([a]) != k([C.encoded_ansatz(11, 2, np.random.default_rng(1))])     # qubit count
    assert k([a]) != k([a, b])                                                    # batch size
    assert k([a]) != tuning.structure_key("batch", [a], device="dev1")            # device
    assert k([a]) != k([a], extra="rows2")
    moved = C.Circuit(a.n, list(a.ops), a.params)
    op = moved.ops[-1]
    moved.ops[-1] = C.Op(op.kind, tuple((t + 1) % a.n for t in op.targets), op.controls, op.params)
    assert k([a]) != k([moved])                                                   # a target


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = tuning.TuneCache(path)
    assert c.get("x") is None
    c.put("x", {"config": {"tile_bits": 12, "threads": 256, "reg_min_bits": 8, "wg_per_cu": 0}})
    c2 = tuning.TuneCache(path)
    assert c2.get("x")["config"]["tile_bits"] == 12
    with open(path) as f:
        assert "x" in json.load(f)
    # a corrupt file is treated as empty
    with open(path, "w") as f:
        f.write("{not json")
    assert tuning.TuneCache(path).get("x") is None
