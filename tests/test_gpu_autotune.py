"""GPU parity of every launch shape the autotuners choose from, and of the
autotuners themselves.

* Batched launch: each tile width (10..14 qubits), thread count (256, 512,
  1024), register-phase threshold, workgroups-per-CU setting, run length
  and phase arithmetic (gate by gate, fused FP32, fused BF16x3) gives the oracle's
  <Z_i> for a batch whose circuits are narrower and wider than the tile (so
  10-qubit tiles cut 11..16-qubit circuits into passes over the arena).
  Tolerance as the other batch tests: the plan's rounding-error bound
  (``errmodel.plan_z_bound``, which depends on its phase arithmetic and its
  number of fused phases and one-by-one gates per circuit).
* The batch autotuner returns a configuration it ran, whose output agreed
  with the default's, and that is the fastest such trial.
* The fusion autotuner's choice, applied, gives the oracle's state.
"""

import numpy as np
import pytest

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod
from paper_2511_19291_amd import tuning
from tests import errmodel

pytestmark = pytest.mark.gpu



def _workload():
    rng = np.random.default_rng(21)
    circuits = [C.encoded_ansatz(n, 2, rng) for n in (4, 9, 10, 11, 13, 16)]
    circuits.append(C.random_circuit(12, 120, 5))     # controls and two-qubit kinds
    circuits.append(C.random_circuit(15, 120, 6))
    return circuits


_ORACLE = {}


def _expected(circuits):
    key = id(circuits)
    if key not in _ORACLE:
        _ORACLE[key] = [oracle.expval_z_all(oracle.run(c), c.n)[0] for c in circuits]
    return _ORACLE[key]


WORK = _workload()

# (tile_bits, threads, reg_min_bits, wg_per_cu, phase_mode, fuse_min_gates, run_bits)
CONFIGS = [(tb, th, 12, 0, pm, 3, 4) for tb in (10, 11, 12, 13, 14) for th in (256, 512, 1024) for pm in (0, 1)]
CONFIGS += [(14, 1024, 4, 0, 1, 1, 4), (14, 256, 8, 0, 1, 1, 6), (12, 512, 15, 0, 1, 3, 5), (10, 256, 10, 2, 1, 2, 3),
            (13, 512, 12, 1, 0, 3, 6), (14, 1024, 12, 0, 2, 1, 3), (11, 512, 9, 0, 2, 2, 5), (12, 256, 4, 0, 1, 64, 4),
            (10, 1024, 12, 0, 1, 3, 5), (14, 512, 12, 0, 1, 3, 3)]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: "tb{}_th{}_reg{}_wg{}_pm{}_fm{}_rb{}".format(*c))
def test_batch_config_parity(sv, cfg):
    d = dict(zip(("tile_bits", "threads", "reg_min_bits", "wg_per_cu", "phase_mode", "fuse_min_gates", "run_bits"),
                 cfg))
    plan = svmod.BatchPlan(WORK, config=d)
    info = plan.info()
    assert info["config"]["tile_bits"] == cfg[0] and info["config"]["threads"] == cfg[1]
    assert info["config"]["phase_mode"] == cfg[4] and info["config"]["fuse_min_gates"] == cfg[5]
    assert info["config"]["run_bits"] == cfg[6]
    assert info["config"]["wg_per_cu"] >= 1 and info["grid"] >= 1
    out = plan.run()
    tol = errmodel.plan_z_bound(plan)
    for i, (c, z) in enumerate(zip(WORK, _expected(WORK))):
        np.testing.assert_allclose(out[i, : c.n], z, atol=tol, err_msg=f"circuit {i} n={c.n} cfg={cfg}")
        assert np.all(out[i, c.n:] == 0)
    plan.free()


def test_bad_batch_config_rejected(sv):
    for bad in ({"tile_bits": 9, "threads": 1024, "reg_min_bits": 12, "wg_per_cu": 0},
                {"tile_bits": 12, "threads": 384, "reg_min_bits": 12, "wg_per_cu": 0},
                {"tile_bits": 12, "threads": 256, "reg_min_bits": 3, "wg_per_cu": 0},
                {"tile_bits": 12, "threads": 256, "reg_min_bits": 12, "wg_per_cu": 17},
                {"tile_bits": 12, "threads": 256, "reg_min_bits": 12, "wg_per_cu": 0, "phase_mode": 3},
                {"tile_bits": 12, "threads": 256, "reg_min_bits": 12, "wg_per_cu": 0, "fuse_min_gates": 0},
                {"tile_bits": 10, "threads": 256, "reg_min_bits": 12, "wg_per_cu": 0, "run_bits": 6}):
        with pytest.raises(svmod.SvError):
            svmod.BatchPlan(WORK[:2], config=bad)


def test_batch_autotune_choice(sv, tmp_path):
    best, trials = svmod.batch_autotune(WORK, reps=2)
    assert len(trials) >= 10
    usable = [t for t in trials if t["max_dev"] <= t["tol"]]
    assert all(t["tol"] > 0 for t in trials)
    assert best in [t["config"] for t in usable]
    # staged search: the choice is at least as fast as the default configuration
    default = trials[0]
    chosen = [t for t in usable if t["config"] == best][0]
    assert chosen["ms"] <= default["ms"]
    # the chosen configuration reproduces the oracle
    plan = svmod.BatchPlan(WORK, config=best)
    out = plan.run()
    for i, (c, z) in enumerate(zip(WORK, _expected(WORK))):
        np.testing.assert_allclose(out[i, : c.n], z, atol=errmodel.plan_z_bound(plan))
    # cached: a second lookup does not run the tuner
    path = str(tmp_path / "tune.json")
    a = tuning.tuned_batch_config(WORK, reps=1, path=path)
    b = tuning.tuned_batch_config(WORK, reps=1, path=path)
    assert a == b and tuning.TuneCache(path).get(tuning.structure_key("batch", WORK)) is not None


@pytest.mark.parametrize("n", [8, 14])
def test_fused_autotune_choice_applies(sv, n):
    circ = C.brickwork_u3_cz(n, 4, 3)
    st = sv.State(n)
    best, trials = svmod.fused_autotune(st, circ, modes=(svmod.FUSED_FP32_MFMA, svmod.FUSED_VALU), reps=1)
    assert best["ms"] == min(t["ms"] for t in trials)
    kinds = {(t["max_k"], t["mode"]) for t in trials}
    assert (1, -1) in kinds and (2, svmod.FUSED_VALU) in kinds
    assert ((5, svmod.FUSED_FP32_MFMA) in kinds) == (n >= 10)
    assert all(t["mode"] != svmod.FUSED_BF16X3 for t in trials)
    st.reset()
    if best["mode"] < 0:
        st.run(circ)
    else:
        st.apply_fused(svmod.fuse_plan(circ, best["max_k"]), best["mode"])
    want = oracle.run(circ)
    np.testing.assert_allclose(st.to_numpy()[0], want, atol=2e-5)
