"""GPU parity of the batched persistent launch (uneven circuits, one
hipGraph-captured kernel) against the oracle circuit by circuit, and against
the per-gate form of the same batch.

Tolerance: <Z_i> within the plan's rounding-error bound
(``errmodel.plan_z_bound``: 2 B + B^2 with B the bound on ||dpsi|| from the
most fused phases and one-by-one gates any circuit of the plan runs, in the
plan's phase arithmetic). The default launch fuses register phases of >= 3
gates on FP32 matrix cores; gate-by-gate and BF16x3 phases are checked too.
The tests print the largest deviation next to its bound."""

import numpy as np
import pytest

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod
from tests import errmodel

pytestmark = pytest.mark.gpu


def _check(out, circuits, plan, expected=None):
    tol = errmodel.plan_z_bound(plan)
    worst = 0.0
    for i, c in enumerate(circuits):
        z = expected[i] if expected is not None else oracle.expval_z_all(oracle.run(c), c.n)[0]
        np.testing.assert_allclose(out[i, : c.n], z, atol=tol, err_msg=f"circuit {i} n={c.n}")
        assert np.all(out[i, c.n:] == 0)
        worst = max(worst, float(np.max(np.abs(out[i, : c.n] - z))))
    print(f"max |d<Z>| {worst:.2e} (bound {tol:.2e})")
    return worst


def test_small_uneven_batch_in_lds(sv):
    """Circuits of 1..14 qubits (whole state in LDS), every gate kind with
    controls, in one launch."""
    circuits = [C.random_circuit(n, 60, 100 + n) for n in range(1, 15)]
    circuits += [C.encoded_ansatz(n, 3, np.random.default_rng(n)) for n in (5, 11, 14)]
    plan = svmod.BatchPlan(circuits)
    out = plan.run()
    _check(out, circuits, plan)


def test_large_circuits_in_passes(sv):
    """15..20 qubits: gate lists cut into LDS-tile passes over the state in
    global memory, mixed with small circuits."""
    rng = np.random.default_rng(9)
    circuits = [C.encoded_ansatz(n, 2, rng) for n in (15, 17, 20, 12, 16)]
    circuits.append(C.random_circuit(18, 150, 7))
    circuits.append(C.random_circuit(16, 150, 8))
    plan = svmod.BatchPlan(circuits)
    out = plan.run()
    _check(out, circuits, plan)
    out_pg = plan.run(pergate=True)
    np.testing.assert_allclose(out, out_pg, atol=errmodel.plan_z_bound(plan) + errmodel.pergate_z_bound(circuits))


def test_graph_replay_with_new_parameters(sv):
    """The captured launch re-reads the parameter block: replays with
    changed parameters (and eager work in between) give each time the
    oracle's result; repeated replays with equal parameters are bitwise
    equal."""
    import torch

    rng = np.random.default_rng(3)
    circuits = [C.encoded_ansatz(n, 2, rng) for n in (6, 10, 15)]
    plan = svmod.BatchPlan(circuits)
    dp = plan.pack()
    out = plan.out_buffer()
    results = []
    for rep in range(3):
        newp = [c.params + 0.1 * (rep + 1) for c in circuits]
        dp.copy_(plan.pack(newp))
        plan.launch(dp, out)
        torch.cuda.synchronize()
        res = out.cpu().numpy().copy()
        tol = errmodel.plan_z_bound(plan)
        for i, c in enumerate(circuits):
            z, _ = oracle.expval_z_all(oracle.run(c, params=newp[i]), c.n)
            np.testing.assert_allclose(res[i, : c.n], z, atol=tol)
        results.append(res)
        x = torch.ones(1000, device=dp.device).sum()   # unrelated eager work between replays
        del x
    plan.launch(dp, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), results[-1])


def _golden_batch256():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "batch256.json")) as f:
        g = json.load(f)
    circuits = C.batch_workload(256, 10, 20, 6, 4)
    assert [c.n for c in circuits] == g["n_qubits"]
    return circuits, [np.array(z) for z in g["expval_z"]]


def test_batch_workload_all_256_default_config(sv):
    """The batching workload at its own size (256 circuits of 10..20 qubits,
    encoded inputs, 6 layers; the launch bench.py times) vs the oracle's
    <Z_i> of every circuit (tests/golden/batch256.json, written by
    oracle/make_goldens.py), under the default configuration."""
    circuits, want = _golden_batch256()
    plan = svmod.BatchPlan(circuits)
    _check(plan.run(), circuits, plan, expected=want)
    plan.free()


def test_batch_workload_all_256_tuned_config(sv):
    """The same 256 circuits under the configuration the autotuner picks for
    them (BF16x3 phases on this workload), within that plan's bound."""
    circuits, want = _golden_batch256()
    best, trials = svmod.batch_autotune(circuits, reps=1)
    chosen = [t for t in trials if t["config"] == best][0]
    assert chosen["max_dev"] <= chosen["tol"]
    plan = svmod.BatchPlan(circuits, config=best)
    print(f"tuned config {best}")
    _check(plan.run(), circuits, plan, expected=want)
    plan.free()


@pytest.mark.parametrize("pm", [0, 1, 2], ids=["gates", "fused_fp32", "fused_bf16x3"])
def test_phase_arithmetic_deep_circuits(sv, pm):
    """Deep circuits of 15..20 qubits (the batching workload's 6-layer
    ansatz; random circuits with two-qubit and controlled gates) with every
    register phase fused (fuse_min_gates 1) in each phase arithmetic, vs the
    oracle, each within its plan's bound."""
    rng = np.random.default_rng(31)
    circuits = [C.encoded_ansatz(n, 6, rng) for n in (15, 18, 20)]
    circuits += [C.random_circuit(17, 300, 12), C.random_circuit(20, 300, 13)]
    plan = svmod.BatchPlan(circuits, config={"phase_mode": pm, "fuse_min_gates": 1})
    out = plan.run()
    tol = errmodel.plan_z_bound(plan)
    errs = []
    for i, c in enumerate(circuits):
        z, _ = oracle.expval_z_all(oracle.run(c), c.n)
        errs.append(float(np.max(np.abs(out[i, : c.n] - z))))
    print(f"phase_mode {pm}: max |dZ| per circuit {['%.2e' % e for e in errs]} (bound {tol:.2e}, "
          f"stats {plan.stats()})")
    assert max(errs) <= tol
    plan.free()


def test_batch_rejects_bad_plans(sv):
    with pytest.raises(svmod.SvError):
        svmod.BatchPlan([C.random_circuit(25, 3, 1)])
    bad = C.Circuit(3, [C.Op("rx", (0,), (), (5,))], np.zeros(1))
    with pytest.raises(svmod.SvError):
        svmod.BatchPlan([bad])


def test_wait_that_gives_up_turns_the_circuit_nan(sv):
    """The bounded inter-pass wait: when a tile of any pass after the first
    gives up waiting (forced from the host: limit -1 gives up at once, so
    every kernel still ends normally), the whole circuit's output is NaN, not
    a finite value from an incomplete state; single-pass circuits (the whole
    state in LDS) are unaffected. Restoring the default limit restores the
    oracle's values on the same plan."""
    rng = np.random.default_rng(17)
    circuits = [C.encoded_ansatz(n, 3, rng) for n in (18, 11, 20, 16, 13)]
    plan = svmod.BatchPlan(circuits)
    passes = plan.info()["n_passes"]
    assert passes > 3
    plan.set_spin_limit(-1)
    out = plan.run()
    for i, c in enumerate(circuits):
        if c.n > 14:                                  # wider than the tile: several passes
            assert np.all(np.isnan(out[i])), (i, c.n, out[i, :4])
        else:
            z, _ = oracle.expval_z_all(oracle.run(c), c.n)
            np.testing.assert_allclose(out[i, : c.n], z, atol=errmodel.plan_z_bound(plan))
    plan.set_spin_limit(1 << 24)
    _check(plan.run(), circuits, plan)
    plan.free()
