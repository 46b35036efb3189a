#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (one step): a 30-qubit complex64 state (8 GiB) reset to |0..0>,
20 brickwork layers of random U3 on every qubit plus CZ on alternating
neighbour pairs (600 U3 + 290 CZ, one sweep per gate), then <sum_i Z_i> by
one FP64 reduction sweep. Inputs are seeded and synthetic.

Printed: ONE JSON line with whole-job gates/s, the roofline of the dominant
kernel (the dense one-qubit sweep, timed live with HIP events on the state's
stream over the timed region) against 8 TB/s and against the copy ceiling
measured in the same run, the error of every reported result against the
complex128 oracle's stored values (tests/golden), the fused-MFMA / adjoint /
batched forms as speedups over the plain form on the same GPU (parameter
shift measured on 16 parameters and scaled), and the CPU oracle timed on
bounded samples of this and the other workloads.

Probes for rocprofv3 (short fixed sequences): --pmc-probe (dense gates,
fused blocks of every form, a plain copy of known size), --adjoint-probe
(forward + matrix-core backward at --n qubits, then a copy), --shots-probe,
--batch-probe. --summarize turns rocprofv3 CSV output into the summaries
under profiles/ (no GPU needed).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "HBM GB/s & gates/s, 30q c64 statevector; fused-MFMA & adjoint vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the fused/adjoint/batched comparisons")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-oracle-timings", action="store_true",
                    help="skip the oracle timings of the other workloads (about 40 s of host work)")
    ap.add_argument("--summarize", nargs="+", metavar="ARG",
                    help="print a profile summary from rocprofv3 CSV output and exit (no GPU): "
                         "stats DIR | traffic FETCH_DIR WRITE_DIR KERNEL_REGEX COPY_BYTES [ALG_BYTES] | "
                         "counters DIR [KERNEL_REGEX]")
    ap.add_argument("--pmc-probe", action="store_true")
    ap.add_argument("--shots-probe", action="store_true",
                    help="the shot-sampling part of the bench alone (n-qubit brickwork output state), for profiles")
    ap.add_argument("--batch-probe", action="store_true", help="three launches of the batching workload per "
                    "configuration (default, BF16x3 phases), for counters")
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="one forward + matrix-core adjoint backward of the n-qubit RX/RY ring, for counters")
    return ap.parse_args()


def kernel_source_digest(files=("k_gates.hip", "sv_device.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2511_19291_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(n: int):
    """HBM bytes per launch of the dense one-qubit kernel from the committed
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"dense_gate_{n}q_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_digest") != kernel_source_digest():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def golden(name: str):
    """Stored oracle values (complex128, written by oracle/make_goldens.py)."""
    path = os.path.join(GOLDEN_DIR, name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def error_vs_golden_z(name: str, n: int, z):
    """Largest |<Z_i> - oracle|, |<sum Z> - oracle| and |norm^2 - oracle|."""
    import numpy as np

    g = golden(name)
    if g is None or z is None or g.get("n") != n:
        return None
    want = np.array(g["expval_z"])
    return {"oracle": f"tests/golden/{name}.json (complex128)",
            "max_abs_z_i": float(np.max(np.abs(np.asarray(z[:n]) - want))),
            "abs_sum_z": abs(float(np.sum(z[:n])) - g["sum_z"]),
            "abs_norm2": abs(float(z[n]) - g["norm2"])}


def copy_ceiling(st, stream) -> float:
    """GB/s of a plain copy of the state (read 8 * 2^n bytes, write the same),
    best of three launches, measured with events on the state's stream."""
    import torch

    from paper_2511_19291_amd import sv

    dst = torch.empty_like(st.tensor)
    nbytes = st.tensor.numel() * 8

    def one():
        sv.check(sv.lib().sv_stream_copy(dst.data_ptr(), st.tensor.data_ptr(), nbytes, stream.cuda_stream))

    one()
    ms = min(_timed_ms(one, stream) for _ in range(3))
    del dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms / 1e3) / 1e9


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the state is not "
              "sharded across GPUs", file=sys.stderr)
        return 2

    if args.summarize:
        return summarize(args.summarize)

    import numpy as np
    import torch

    from paper_2511_19291_amd import circuits as C
    from paper_2511_19291_amd import sv

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = args.n

    if args.pmc_probe:
        return run_pmc_probe(n)
    if args.adjoint_probe:
        return run_adjoint_probe(n)
    if args.batch_probe:
        return run_batch_probe()
    if args.shots_probe:
        circ = C.brickwork_u3_cz(n, 20, 2)
        st = sv.State(n)
        print(json.dumps({"shots_probe": shots_extra(st, circ, sv.fuse_plan(circ, 5), stream)}), flush=True)
        return 0

    circ = C.brickwork_u3_cz(n, 20, 2)
    table = sv.OpTable(circ.ops)
    params = np.ascontiguousarray(circ.params)
    # the dominant kernel: dense U3 on targets >= 7 all run k_gate<1, 5, 1, true>
    # (float4 member streams; targets 1..6 take the shuffle form, 0 the pair form)
    dense_ops = [i for i, op in enumerate(circ.ops) if op.kind == "u3" and op.targets[0] >= 7]
    dense_set = set(dense_ops)
    n_gates = len(circ.ops)

    st = sv.State(n)
    last_z = [None]

    def step(events=None):
        st.reset()
        i = 0
        while i < n_gates:
            if events is not None and i in dense_set:
                events[0].append(torch.cuda.Event(enable_timing=True))
                events[1].append(torch.cuda.Event(enable_timing=True))
                events[0][-1].record(stream)
                st.run_ops(table, i, 1, params)
                events[1][-1].record(stream)
                i += 1
            else:
                j = i
                while j < n_gates and (events is None or j not in dense_set):
                    j += 1
                st.run_ops(table, i, j - i, params)
                i = j
        z = st.expval_z_all()[0]
        last_z[0] = z
        return float(np.sum(z[:n]))

    # workgroup order of the one-target dense sweep, chosen per target on this
    # device before anything is timed (identity sweeps: the state is unchanged)
    t_tune = time.perf_counter()
    order_ms = st.reset().tune_sweep_order()
    order_mask = st.sweep_order()
    sweep_order = {"tuned_before_warmup": True, "tune_s": round(time.perf_counter() - t_tune, 3),
                   "xcd_targets": [t for t in range(n) if (order_mask >> t) & 1],
                   "median_ms_hw_xcd": {str(t): [round(float(order_ms[t, 0]), 4), round(float(order_ms[t, 1]), 4)]
                                        for t in range(n) if order_ms[t, 0] > 0}}
    print(f"# warmup {args.warmup} step(s) of {circ.name} ({n_gates} gates)", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = ([], [])
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    sumz = None
    for k in range(args.steps):
        sumz = step(ev)
        print(f"# step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    elapsed_ms = t_start.elapsed_time(t_end)
    ms_per_step = elapsed_ms / args.steps
    gates_per_s = n_gates * args.steps / (elapsed_ms / 1e3)
    dense_ms = [a.elapsed_time(b) for a, b in zip(*ev)]
    avg_dense_ms = float(np.mean(dense_ms))
    alg_bytes = 16.0 * (1 << n)          # read + write every amplitude, complex64
    achieved = alg_bytes / (avg_dense_ms / 1e3) / 1e9
    traffic = read_traffic(n)
    # the measured ceiling: a plain copy of the state (8 * 2^n bytes read, the same written)
    copy_GBps = copy_ceiling(st, stream)
    # algorithmic bytes of the whole step: one sweep per gate (CZ by the
    # 128-byte line rule: both qubits >= 4 -> 4 B/amplitude, one below 4 ->
    # 8, both below 4 -> 16), the reset (8) and the reduction (8)
    counts = circ.counts()
    cz_bytes = 0
    for op in circ.ops:
        if op.kind == "z" and op.controls:
            lo = min(op.targets[0], op.controls[0])
            hi = max(op.targets[0], op.controls[0])
            cz_bytes += 16 if hi < 4 else (8 if lo < 4 else 4)
    step_bytes = (counts.get("u3", 0) * 16 + cz_bytes + 8 + 8) * (1 << n)
    err = error_vs_golden_z("brickwork30", n, last_z[0]) if n == 30 else None
    out = {
        "metric": METRIC,
        "value": round(gates_per_s, 3),
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"brickwork{n}: {n}-qubit complex64 state, 20 layers of U3 on every qubit + CZ on "
                        f"alternating neighbour pairs ({counts.get('u3', 0)} U3 + {counts.get('cz', 0)} CZ, "
                        f"one sweep per gate), then <sum Z_i>",
            "n_qubits": n,
            "gates_per_step": n_gates,
            "state_bytes": 8 * (1 << n),
        },
        "hbm_GBps_step": round(step_bytes / (ms_per_step / 1e3) / 1e9, 1),
        "hbm_frac_of_copy_step": round(step_bytes / (ms_per_step / 1e3) / 1e9 / copy_GBps, 4),
        "copy_GBps": round(copy_GBps, 1),
        "sum_z": sumz,
        "error_vs_oracle": err,
        "wall_s_timed": round(wall, 3),
        "sweep_order": sweep_order,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_gate<1, 5, 1, true> (dense one-qubit sweep, split-halves form, target >= 7)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "frac_of_copy": round(achieved / copy_GBps, 4),
            "copy_GBps": round(copy_GBps, 1),
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_ms": round(avg_dense_ms, 4),
            "launches_timed": len(dense_ms),
        },
    }
    st.free()
    del st
    torch.cuda.empty_cache()

    if not args.no_extras:
        out.update(extras(args, n, gates_per_s, avg_dense_ms, copy_GBps))

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(circ, args.cpu_seconds)
        if not args.no_oracle_timings:
            out["oracle_timings"] = oracle_timings()
    print(json.dumps(out), flush=True)
    return 0


def _timed_ms(fn, stream) -> float:
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def extras(args, n, plain_gates_per_s, avg_dense_ms, copy_GBps) -> dict:
    """Fused-MFMA, adjoint and batched forms against the plain form, each on
    its own workload, all on this GPU."""
    import numpy as np
    import torch

    from paper_2511_19291_amd import circuits as C
    from paper_2511_19291_amd import sv

    stream = torch.cuda.current_stream()
    res = {}

    # -- one dense U3 sweep on every target of the n-qubit state (16 B per
    # amplitude each), four launches per target after one untimed
    st = sv.State(n)
    st.reset()
    per_t = []
    for t in range(n):
        b = C._Builder(n)
        b.gate("u3", [t], values=[0.3 + 0.1 * t, 1.1, 2.3])
        c1 = b.build(f"u3_t{t}")
        tab = sv.OpTable(c1.ops)
        p1 = np.ascontiguousarray(c1.params)
        st.run_ops(tab, 0, 1, p1)
        ms = _timed_ms(lambda: [st.run_ops(tab, 0, 1, p1) for _ in range(4)], stream) / 4
        per_t.append(16 * (1 << n) / (ms / 1e3) / 1e9)
    st.free()
    del st
    torch.cuda.empty_cache()
    srt = sorted(per_t)
    res["per_target_u3"] = {
        "workload": f"one U3 sweep of the {n}-qubit complex64 state on each target 0..{n - 1}; 16 B/amplitude",
        "GBps": [round(x, 1) for x in per_t],
        "min_GBps": round(srt[0], 1), "median_GBps": round(srt[len(srt) // 2], 1),
        "min_frac_of_8TBps": round(srt[0] / 8000.0, 3), "median_frac_of_8TBps": round(srt[len(srt) // 2] / 8000.0, 3),
        "min_frac_of_copy": round(srt[0] / copy_GBps, 3), "median_frac_of_copy": round(srt[len(srt) // 2] / copy_GBps, 3),
        "argmin_target": int(np.argmin(per_t)),
    }

    # -- fused blocks: the same 30-qubit brickwork, and the 32-qubit instance
    fused = {}
    for nq, seed, with_plain in ((n, 2, False), (32, 3, True)):
        circ = C.brickwork_u3_cz(nq, 20, seed)
        t0 = time.perf_counter()
        blocks = sv.fuse_plan(circ, 5)
        plan_ms = (time.perf_counter() - t0) * 1e3
        st = sv.State(nq)
        entry = {"gates": len(circ.ops), "blocks": len(blocks), "plan_ms": round(plan_ms, 2)}
        zs = {}
        for mode, name in ((sv.FUSED_FP32_MFMA, "fp32_mfma"), (sv.FUSED_BF16X3, "bf16x3")):
            st.reset()
            st.apply_fused(blocks[:2], mode)
            ms = _timed_ms(lambda: (st.reset(), st.apply_fused(blocks, mode)), stream)
            per_block = ms / len(blocks)
            gbps = 16 * (1 << nq) / (per_block / 1e3) / 1e9
            entry[name] = {"ms": round(ms, 2), "gates_per_s": round(len(circ.ops) / (ms / 1e3), 1),
                           "ms_per_block": round(per_block, 4),
                           "GBps_per_block": round(gbps, 1), "frac_of_copy_per_block": round(gbps / copy_GBps, 3),
                           "TFLOPs_per_block": round(8 * 32 * (1 << nq) / (per_block / 1e3) / 1e12, 2)}
            zs[name] = st.expval_z_all()[0]          # the state holds this mode's output
            if nq == 30:
                entry[name]["error_vs_oracle"] = error_vs_golden_z("brickwork30", nq, zs[name])
        # six-qubit blocks off qubits 0..5 (BF16x3 only), five-qubit blocks elsewhere
        blocks6 = sv.fuse_plan(circ, 6)
        st.reset()
        st.apply_fused(blocks6[:2], sv.FUSED_BF16X3)
        ms6 = _timed_ms(lambda: (st.reset(), st.apply_fused(blocks6, sv.FUSED_BF16X3)), stream)
        entry["bf16x3_k6"] = {"blocks": len(blocks6), "six_qubit_blocks": sum(len(t) == 6 for t, _ in blocks6),
                              "ms": round(ms6, 2), "gates_per_s": round(len(circ.ops) / (ms6 / 1e3), 1),
                              "ms_per_block": round(ms6 / len(blocks6), 4)}
        zs["bf16x3_k6"] = st.expval_z_all()[0]
        if nq == 30:
            entry["bf16x3_k6"]["error_vs_oracle"] = error_vs_golden_z("brickwork30", nq, zs["bf16x3_k6"])
        if with_plain:
            table = sv.OpTable(circ.ops)
            p = np.ascontiguousarray(circ.params)
            ms = _timed_ms(lambda: (st.reset(), st.run_ops(table, 0, len(circ.ops), p)), stream)
            entry["plain_ms"] = round(ms, 2)
            zp = st.expval_z_all()[0]
            # no oracle state at 32 qubits (32 GiB of complex64, 64 GiB in complex128): against the plain sweeps
            for name in ("fp32_mfma", "bf16x3", "bf16x3_k6"):
                entry[name]["max_abs_z_i_vs_plain"] = float(np.max(np.abs(zs[name][:nq] - zp[:nq])))
        else:
            entry["plain_ms"] = round(len(circ.ops) / plain_gates_per_s * 1e3, 2)
        for name in ("fp32_mfma", "bf16x3", "bf16x3_k6"):
            entry[name]["speedup_vs_plain"] = round(entry["plain_ms"] / entry[name]["ms"], 2)
        if nq == n:
            # fusion width and arithmetic picked by the library's autotuner
            # (plain sweeps, vector blocks of k = 2..5, matrix-core blocks)
            t0 = time.perf_counter()
            best, trials = sv.fused_autotune(st, circ, modes=(sv.FUSED_FP32_MFMA, sv.FUSED_BF16X3, sv.FUSED_VALU),
                                             reps=1)
            names = {-1: "plain", sv.FUSED_FP32_MFMA: "fp32_mfma", sv.FUSED_BF16X3: "bf16x3", sv.FUSED_VALU: "valu"}
            entry["autotune"] = {
                "chosen": {"max_k": best["max_k"], "mode": names[best["mode"]], "ms": round(best["ms"], 2),
                           "sweeps": best["n_sweeps"]},
                "trials": [{"max_k": t["max_k"], "mode": names[t["mode"]], "sweeps": t["n_sweeps"],
                            "ms": round(t["ms"], 2)} for t in trials],
                "tune_s": round(time.perf_counter() - t0, 2),
            }
        fused[f"brickwork{nq}"] = entry
        if nq == n:
            res["shots"] = shots_extra(st, circ, blocks, stream)
        st.free()
        del st
        torch.cuda.empty_cache()
        print(f"# fused {nq}q done", file=sys.stderr, flush=True)
    res["fused"] = fused

    # -- adjoint backward on the 28-qubit RX/RY + CNOT-ring ansatz
    circ = C.rxry_ring(28, 10, 5)
    terms = C.z_sum_terms(28)
    st = sv.State(28)
    table = sv.OpTable(circ.ops)
    p = np.ascontiguousarray(circ.params)
    fwd_ms = _timed_ms(lambda: (st.reset(), st.run_ops(table, 0, len(circ.ops), p)), stream)
    t0 = time.perf_counter()
    loss, grad, drift = st.adjoint_grad(circ, terms)
    bwd_ms = (time.perf_counter() - t0) * 1e3
    st.reset()
    st.run_ops(table, 0, len(circ.ops), p)
    t0 = time.perf_counter()
    loss, grad, drift = st.adjoint_grad(circ, terms)
    bwd_ms = min(bwd_ms, (time.perf_counter() - t0) * 1e3)
    # blocked backward: one sweep per block of gates on 3, 4 or 5 qubits
    blocked = {}
    for lb in (3, 4, 5, sv.ADJOINT_MFMA):
        st.reset()
        st.run_ops(table, 0, len(circ.ops), p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss_b, grad_b, drift_b = st.adjoint_grad(circ, terms, block_qubits=lb)
        ms_b = (time.perf_counter() - t0) * 1e3
        if lb == sv.ADJOINT_MFMA:
            grad_mfma = grad_b[0].copy()
        blocked["mfma4" if lb == sv.ADJOINT_MFMA else f"block{lb}"] = {"backward_ms": round(ms_b, 2), "backward_over_forward": round(ms_b / fwd_ms, 3),
                                 "max_grad_diff_vs_per_gate": float(np.max(np.abs(grad_b[0] - grad[0]))),
                                 "drift": float(drift_b[0])}
    # the autograd layers' forward: row-shared gates fused into 5-qubit
    # matrix-core blocks (host planning included in the time)
    fwd_fused_ms = min(_timed_ms(lambda: (st.reset(), st.run_fused(circ)), stream) for _ in range(2))
    n_par = circ.n_params
    # parameter shift measured on the GPU for 16 seeded parameters (two
    # forwards and one <Z> reduction each), scaled to all parameters; once
    # with plain sweeps, once with the fused forward
    which = np.random.default_rng(28).choice(n_par, size=16, replace=False)
    shift = {}
    for fwd in ("plain", "fused"):
        vals = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in which:
            pair = []
            for sgn in (1.0, -1.0):
                prm = circ.params.copy()
                prm[q] += sgn * np.pi / 2
                st.reset()
                if fwd == "plain":
                    st.run_ops(table, 0, len(circ.ops), np.ascontiguousarray(prm))
                else:
                    st.run_fused(circ, prm)
                pair.append(float(np.sum(st.expval_z_all()[0][:28])))
            vals.append(0.5 * (pair[0] - pair[1]))
        ms16 = (time.perf_counter() - t0) * 1e3
        shift[fwd] = {"ms_16_params": round(ms16, 1), "ms_scaled_to_all": round(ms16 / 16 * n_par, 1),
                      "max_abs_vs_adjoint": float(np.max(np.abs(np.array(vals) - grad[0][which])))}
    shift_ms = shift["fused"]["ms_scaled_to_all"]
    # the autograd layers' default backward at this width: matrix-core blocks
    default_ms = blocked["mfma4"]["backward_ms"]
    res["adjoint"] = {
        "workload": "rxry_ring28: 28 qubits, 10 x [RX all, RY all, CNOT ring], loss <sum Z_i>",
        "params": n_par, "forward_ms": round(fwd_ms, 2), "forward_fused_ms": round(fwd_fused_ms, 2),
        "train_step_ms": round(fwd_fused_ms + blocked["mfma4"]["backward_ms"], 2),
        "backward_ms": round(default_ms, 2),
        "backward_kind": "matrix-core blocks of 4 qubits (the autograd default from 13 qubits)",
        "backward_over_forward": round(default_ms / fwd_ms, 3),
        "backward_per_gate_ms": round(bwd_ms, 2), "per_gate_over_forward": round(bwd_ms / fwd_ms, 3),
        "param_shift": {"measured": "16 seeded parameters on this GPU, two forwards + <sum Z> each, "
                                    "scaled to all parameters", "plain_forward": shift["plain"],
                        "fused_forward": shift["fused"]},
        "speedup_vs_param_shift": round(shift_ms / default_ms, 1),
        "speedup_basis": "parameter shift with the fused forward (scaled from 16 parameters) / matrix-core backward",
        # gate-equivalent bytes of the per-gate adjoint (32 B/amplitude per
        # rotation, 16 per CNOT) over the matrix-core backward's time: an
        # effective rate, not an HBM fraction
        "backward_effective_GBps": round(sum(16 if op.controls else 32 for op in circ.ops) * (1 << 28)
                                         / (default_ms / 1e3) / 1e9, 1),
        "loss": float(loss[0]), "grad_norm": float(np.linalg.norm(grad[0])), "drift": float(drift[0]),
        "blocked": blocked,
    }
    g28 = golden("ring28")
    if g28 is not None:
        want = np.array(g28["grad"])
        res["adjoint"]["error_vs_oracle"] = {
            "oracle": "tests/golden/ring28.json (complex128 adjoint)",
            "loss_abs": abs(float(loss[0]) - g28["loss"]),
            "per_gate_rel_max": float(np.max(np.abs(grad[0] - want)) / np.max(np.abs(want))),
            "mfma4_rel_max": float(np.max(np.abs(grad_mfma - want)) / np.max(np.abs(want))),
        }
    st.free()
    del st
    torch.cuda.empty_cache()
    print("# adjoint done", file=sys.stderr, flush=True)

    # -- the paper's profiling workload: RY encoding + 3 x [CNOT ring, RY],
    #    batch 16, Adam on the inputs; 5 iterations, the last one timed
    prof = {}
    from paper_2511_19291_amd.autograd import MeasureAllZ
    for nq in (18, 24):
        circ, rows = C.profiling_ladder(nq, 3, 16, seed=7)
        layer = MeasureAllZ(circ, 16)
        x = torch.tensor(rows[:, :nq].copy(), dtype=torch.float64, requires_grad=True)
        theta = torch.tensor(rows[:, nq:])
        opt = torch.optim.Adam([x], lr=0.05)
        losses, times = [], []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            opt.zero_grad()
            loss = layer(torch.cat([x, theta], dim=1)).abs().sum()
            loss.backward()
            opt.step()
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            losses.append(loss.item())
        prof[f"n{nq}"] = {"gates": len(circ.ops), "batch": 16, "final_step_ms": round(times[-1], 2),
                          "median_step_ms": round(float(np.median(times)), 2),
                          "loss_first": round(losses[0], 6), "loss_last": round(losses[-1], 6),
                          "state_bytes": 16 * 8 * (1 << nq), "adjoint_buffer_bytes": 16 * 8 * (1 << nq)}
        layer.state.free()
        del layer
        torch.cuda.empty_cache()
    res["profiling_ladder"] = {
        "workload": "paper's profiling ansatz: RY(x) encoding, 3 x [CNOT ring, RY(theta)], batch 16, "
                    "loss sum |<Z_i>|, Adam (lr 0.05) on the inputs, 5 iterations; times are wall ms per "
                    "iteration (forward + adjoint backward + optimizer step)",
        **prof,
    }
    print("# profiling ladder done", file=sys.stderr, flush=True)

    # -- batched: 256 uneven circuits in one graph launch vs per-gate launches;
    #    the launch shape is picked by the library's autotuner
    circs = C.batch_workload(256, 10, 20, 6, 4)
    t0 = time.perf_counter()
    best, trials = sv.batch_autotune(circs, reps=2)
    tune_s = time.perf_counter() - t0
    timings, outs, stats = {}, {}, {}
    modes = (("default", None), ("tuned", best), ("gate_by_gate", {"phase_mode": 0}),
             ("fused_fp32", {"phase_mode": 1}), ("fused_bf16x3", {"phase_mode": 2}))
    for name, cfg in modes:
        plan = sv.BatchPlan(circs, config=cfg)
        dp = plan.pack()
        out = plan.out_buffer()
        plan.launch(dp, out)
        torch.cuda.synchronize()
        timings[name] = min(_timed_ms(lambda: plan.launch(dp, out), stream) for _ in range(3))
        outs[name] = out.cpu().numpy().copy()
        stats[name] = plan.stats()
        if name == "tuned":
            info = plan.info()
            t0 = time.perf_counter()
            plan.launch(dp, out, pergate=True)
            torch.cuda.synchronize()
            pergate_ms = (time.perf_counter() - t0) * 1e3
        plan.free()
    graph_ms = timings["tuned"]
    gates = sum(len(c.ops) for c in circs)

    def mode_entry(name, flop_per_amp, peak):
        st = stats[name]
        e = {"ms": round(timings[name], 3), "gates_per_s": round(gates / (timings[name] / 1e3), 1),
             "max_dev_vs_default": float(np.max(np.abs(outs[name] - outs["default"]))),
             "fused_phases": st["n_fused_phases"], "phases": st["n_phases"], "passes": st["n_passes"]}
        if flop_per_amp:
            # matrix-core work of the fused phases over the whole launch
            tf = st["fused_amp_phases"] * flop_per_amp / (timings[name] / 1e3) / 1e12
            e["mfma_TFLOPs"] = round(tf, 1)
            e["mfma_peak_TFLOPs"] = peak
            e["mfma_frac"] = round(tf / peak, 3)
        return e

    res["batched"] = {
        "workload": "256 circuits, n uniform in 10..20, encoded RY inputs + 6 x [RY, RZ, CNOT ladder], all <Z_i>",
        "gates": gates, "graph_launch_ms": round(graph_ms, 3), "per_gate_launches_ms": round(pergate_ms, 2),
        "gates_per_s": round(gates / (graph_ms / 1e3), 1),
        "speedup_vs_per_gate": round(pergate_ms / graph_ms, 2),
        "default_config_ms": round(timings["default"], 3),
        # a fused phase amplitude costs, FP32 (Gauss): three real 16-wide
        # rows = 48 multiply-adds = 96 FLOP; BF16x3: three rows of the real
        # 32x32 form, 3 x 64 multiply-adds = 384 FLOP
        "phase_arithmetic": {"gate_by_gate": mode_entry("gate_by_gate", 0, None),
                             "fused_fp32": mode_entry("fused_fp32", 96, 157.3),
                             "fused_bf16x3": mode_entry("fused_bf16x3", 3 * 128, 2500.0)},
        "autotune": {"chosen": info["config"], "grid": info["grid"], "tasks": info["n_tasks"],
                     "passes": info["n_passes"], "configs_tried": len(trials), "tune_s": round(tune_s, 2)},
    }
    gb = golden("batch256")
    if gb is not None and gb["n_qubits"] == [c.n for c in circs]:
        def zerr(o):
            return float(max(np.max(np.abs(o[i, : c.n] - np.array(gb["expval_z"][i]))) for i, c in enumerate(circs)))
        res["batched"]["error_vs_oracle"] = {"oracle": "tests/golden/batch256.json (complex128)",
                                             **{f"max_abs_z_i_{k}": zerr(outs[k]) for k in outs}}
    print("# batched done", file=sys.stderr, flush=True)
    return res


def shots_extra(st, circ, blocks, stream) -> dict:
    """Shot noise (Sec. 4.3) on the 30-qubit brickwork output state: 2^20
    exact draws (inverse CDF) and one Gaussian histogram of 10^9 shots
    (all 2^n bins)."""
    import numpy as np
    import torch

    from paper_2511_19291_amd import sv

    n = st.n
    st.reset()
    st.apply_fused(blocks, sv.FUSED_FP32_MFMA)
    rng = np.random.default_rng(41)
    nshots = 1 << 20
    u = torch.as_tensor(rng.random(nshots), device=st.tensor.device)
    st.sample_exact(u)
    exact_ms = min(_timed_ms(lambda: st.sample_exact(u), stream) for _ in range(3))
    g = torch.Generator(device=st.tensor.device)
    g.manual_seed(5)
    z = torch.randn(1 << n, dtype=torch.float64, device=st.tensor.device, generator=g)
    y = st.sample_gaussian(z, 1e9)
    gauss_ms = min(_timed_ms(lambda: st.sample_gaussian(z, 1e9), stream) for _ in range(3))
    ysum = float(y.sum())
    del y, z, u
    torch.cuda.empty_cache()
    print("# shots done", file=sys.stderr, flush=True)
    return {
        "workload": f"{n}-qubit brickwork output state (fused FP32), exact: {nshots} draws; "
                    "gaussian: 1e9 shots over all 2^n bins",
        "exact_ms": round(exact_ms, 3), "exact_shots_per_s": round(nshots / (exact_ms / 1e3), 1),
        # the mass sweep reads every amplitude once; each draw reads its chunk of 128
        "exact_alg_GBps": round((8 * (1 << n) + 1024 * nshots) / (exact_ms / 1e3) / 1e9, 1),
        "exact_frac_of_8TBps": round((8 * (1 << n) + 1024 * nshots) / (exact_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 3),
        "gaussian_ms": round(gauss_ms, 3),
        "gaussian_alg_GBps": round(40 * (1 << n) / (gauss_ms / 1e3) / 1e9, 1),
        "gaussian_sum_minus_shots": ysum - 1e9,
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(circ, seconds: float) -> dict:
    """The CPU oracle, as it is, on a bounded sample of the same workload: the
    same n-qubit complex128 state and the circuit's first gates, as many as
    fit in about ``seconds`` (at least 3)."""
    import numpy as np

    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    n = circ.n
    t0 = time.perf_counter()
    psi = oracle.basis_state(n, 0)
    t_init = time.perf_counter() - t0
    done = 0
    t1 = time.perf_counter()
    while done < len(circ.ops):
        oracle.apply_op(psi, n, circ.ops[done], circ.params)
        done += 1
        if done >= 3 and time.perf_counter() - t1 > seconds:
            break
    dt = time.perf_counter() - t1
    del psi
    return {
        "value": round(done / dt, 4),
        "unit": "gates/s",
        "cores": threads,
        "cpu_model": _cpu_model(),
        "kind": "oracle",
        "sample": f"first {done} gates of the {n}-qubit workload on a complex128 state "
                  f"({dt:.1f} s; state init {t_init:.1f} s not counted)",
    }


_C1_ONE_CORE = """
import sys, time
sys.path.insert(0, {root!r})
import oracle
from paper_2511_19291_amd import circuits as C
c = C.WORKLOADS["hea12"]()
ts = []
for _ in range(3):
    t0 = time.perf_counter()
    oracle.expval_z_all(oracle.run(c), 12)
    ts.append(time.perf_counter() - t0)
print(sorted(ts)[1] * 1e3)
"""


def oracle_timings(budget_s: float = 6.0) -> dict:
    """The CPU oracle, as it is, on the other workloads, each on a bounded
    sample (the entry says what it covers) so the whole takes well under a
    minute: C1 (12-qubit ansatz, full state and <Z>) on all cores and on one
    (a child process with OMP_NUM_THREADS=1; nothing there touches the GPU),
    the 24-qubit fusion instance gate by gate, the batching workload circuit
    by circuit, the 14-qubit differentiation copy's parameter-shift and
    central-difference gradients (all 280 parameters), and the 28-qubit
    forward."""
    import subprocess

    import numpy as np

    import oracle
    from paper_2511_19291_amd import circuits as C

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    out = {"kind": "oracle", "cores": threads, "cpu_model": _cpu_model()}

    c1 = C.WORKLOADS["hea12"]()
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.expval_z_all(oracle.run(c1), 12)
        ts.append(time.perf_counter() - t0)
    one = None
    try:
        r = subprocess.run([sys.executable, "-c", _C1_ONE_CORE.format(root=ROOT)], capture_output=True, text=True,
                           timeout=120, env={**os.environ, "OMP_NUM_THREADS": "1"})
        one = float(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        one = None
    out["c1_hea12"] = {"gates": len(c1.ops), "ms_all_cores": round(sorted(ts)[1] * 1e3, 3),
                       "ms_one_core": None if one is None else round(one, 3),
                       "sample": "whole circuit and <Z_i>, median of 3"}

    def gates_sample(circ, label):
        psi = oracle.basis_state(circ.n, 0)
        done = 0
        t0 = time.perf_counter()
        while done < len(circ.ops) and (done < 3 or time.perf_counter() - t0 < budget_s):
            oracle.apply_op(psi, circ.n, circ.ops[done], circ.params)
            done += 1
        dt = time.perf_counter() - t0
        del psi
        return {"gates_per_s": round(done / dt, 3), "gates_done": done, "gates": len(circ.ops),
                "s_whole_circuit_est": round(len(circ.ops) * dt / done, 1),
                "sample": f"first {done} of {len(circ.ops)} gates of {label} ({dt:.1f} s)"}

    out["c3_fused24"] = gates_sample(C.WORKLOADS["fused24"](), "the 24-qubit fusion instance")
    circs = C.batch_workload(256, 10, 20, 6, 4)
    done = 0
    t0 = time.perf_counter()
    while done < len(circs) and (done < 1 or time.perf_counter() - t0 < 2.5 * budget_s):
        c = circs[done]
        oracle.expval_z_all(oracle.run(c), c.n)
        done += 1
    dt = time.perf_counter() - t0
    out["c4_batch256"] = {"circuits_done": done, "s": round(dt, 2),
                          "s_all_256_est": round(dt if done == len(circs) else
                                                 dt * sum(len(c.ops) << c.n for c in circs) /
                                                 sum(len(c.ops) << c.n for c in circs[:done]), 1),
                          "sample": f"the first {done} of 256 circuits in order, whole state and <Z_i> each "
                                    "(the estimate scales by gates x 2^n)"}
    c14 = C.WORKLOADS["ring14"]()
    terms = C.z_sum_terms(14)
    t0 = time.perf_counter()
    g_shift = oracle.grad_param_shift(c14, terms)
    t_shift = time.perf_counter() - t0
    t0 = time.perf_counter()
    g_fd = oracle.grad_finite_diff(c14, terms)
    t_fd = time.perf_counter() - t0
    out["c5_ring14"] = {"params": c14.n_params, "param_shift_s": round(t_shift, 2), "finite_diff_s": round(t_fd, 2),
                        "max_abs_shift_minus_fd": float(np.max(np.abs(g_shift - g_fd))),
                        "sample": "every parameter, both rules"}
    out["c5_ring28_forward"] = gates_sample(C.WORKLOADS["ring28"](), "the 28-qubit differentiation forward")
    return out


def _csvs(d: str, suffix: str):
    import glob

    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    import csv

    rows = []
    for f in files:
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, regex=None):
    """{(kernel, dispatch): {counter: value summed over dimensions}, duration ms}"""
    import re

    vals, dur = {}, {}
    for r in rows:
        name = r["Kernel_Name"]
        if regex and not re.search(regex, name):
            continue
        key = (name, int(r["Dispatch_Id"]))
        vals.setdefault(key, {})
        vals[key][r["Counter_Name"]] = vals[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        dur[key] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    return vals, dur


def summarize(argv) -> int:
    """Profile summaries from rocprofv3 CSV output (no GPU needed):
      stats DIR                       kernel statistics (--kernel-trace --stats)
      traffic FETCH_DIR WRITE_DIR RE COPY_BYTES [ALG_BYTES]
                                      FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the kernels
                                      matching RE, scaled by COPY_BYTES / what the same counter reads
                                      for the plain copy kernel k_copy of the same run
      counters DIR [RE]               per kernel: median duration, launch shape and counters; with
                                      GRBM_GUI_ACTIVE the clock (busy cycles / 8 XCDs / duration),
                                      with SQ_VALU_MFMA_BUSY_CYCLES the matrix cores' busy share, and
                                      with SQ_WAVE_CYCLES the shares of wave time at a wait
                                      (SQ_WAIT_ANY) and waiting to issue (SQ_WAIT_INST_ANY)"""
    import statistics

    kind = argv[0]
    if kind == "stats":
        rows = _csvs(argv[1], "kernel_stats.csv")
        print("rocprofv3 kernel statistics (durations in microseconds):\n")
        print(" calls     avg_us     min_us     max_us   total_ms    pct  kernel")
        for r in rows:
            print(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} {float(r['MinNs']) / 1e3:10.1f} "
                  f"{float(r['MaxNs']) / 1e3:10.1f} {float(r['TotalDurationNs']) / 1e6:10.2f} "
                  f"{float(r['Percentage']):6.2f}  {r['Name'][:140]}")
        return 0
    if kind == "traffic":
        import re

        fetch_dir, write_dir, regex, copy_bytes = argv[1], argv[2], argv[3], float(argv[4])
        alg = float(argv[5]) if len(argv) > 5 else None
        got = {}
        for ctr, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
            vals, _ = _per_dispatch(_csvs(d, "counter_collection.csv"))
            copy = [v[ctr] for (k, _), v in vals.items() if "k_copy" in k and ctr in v]
            kern = [v[ctr] for (k, _), v in vals.items() if re.search(regex, k) and ctr in v]
            if not copy or not kern:
                raise SystemExit(f"{ctr}: no k_copy or no dispatch matching {regex!r} in {d}")
            got[ctr] = (statistics.mean(copy), statistics.mean(kern), len(kern))
        fscale = copy_bytes / (got["FETCH_SIZE"][0] * 1024)
        wscale = copy_bytes / (got["WRITE_SIZE"][0] * 1024)
        rd = got["FETCH_SIZE"][1] * 1024 * fscale
        wr = got["WRITE_SIZE"][1] * 1024 * wscale
        print("FETCH_SIZE and WRITE_SIZE are KiB per dispatch; each is scaled by known copy bytes / what the same")
        print("counter reads for the copy kernel (k_copy) of the same run.\n")
        print(f"copy bytes each way: {copy_bytes:.0f}")
        print(f"copy FETCH_SIZE KiB: {got['FETCH_SIZE'][0]:.1f}")
        print(f"copy WRITE_SIZE KiB: {got['WRITE_SIZE'][0]:.1f}")
        print(f"fetch_scale: {fscale:.4f}")
        print(f"write_scale: {wscale:.4f}")
        print(f"kernel dispatches (fetch run, write run): {got['FETCH_SIZE'][2]}, {got['WRITE_SIZE'][2]}")
        print(f"kernel FETCH_SIZE KiB (mean): {got['FETCH_SIZE'][1]:.1f}")
        print(f"kernel WRITE_SIZE KiB (mean): {got['WRITE_SIZE'][1]:.1f}")
        print(f"read_bytes_per_launch: {rd:.0f}")
        print(f"write_bytes_per_launch: {wr:.0f}")
        print(f"traffic_bytes_per_launch: {rd + wr:.0f}")
        if alg:
            print(f"alg_bytes_per_launch: {alg:.0f}")
            print(f"traffic_over_alg: {(rd + wr) / alg:.4f}")
        return 0
    if kind == "counters":
        regex = argv[2] if len(argv) > 2 else None
        rows = _csvs(argv[1], "counter_collection.csv")
        vals, dur = _per_dispatch(rows, regex)
        meta = {}
        for r in rows:
            meta.setdefault(r["Kernel_Name"], {k: r.get(k, "") for k in ("Workgroup_Size", "LDS_Block_Size",
                                                                            "VGPR_Count", "Accum_VGPR_Count")})
        by = {}
        for key, v in vals.items():
            by.setdefault(key[0], []).append((dur[key], v))
        for name, lst in by.items():
            med = lambda xs: sorted(xs)[len(xs) // 2]
            ms = med([x[0] for x in lst])
            ctrs = sorted({c for _, v in lst for c in v})
            print(f"{name[:120]}")
            print(f"  dispatches {len(lst)}, median duration {ms:.4f} ms")
            m = meta.get(name, {})
            if m.get("VGPR_Count"):
                print(f"  launch: workgroup {m['Workgroup_Size']} threads, LDS {m['LDS_Block_Size']} B, "
                      f"rocprofv3 VGPR_Count {m['VGPR_Count']} / Accum_VGPR_Count {m['Accum_VGPR_Count']}")
            for c in ctrs:
                print(f"  {c:28s} median {med([v.get(c, 0.0) for _, v in lst]):.4e}")
            if "SQ_WAVE_CYCLES" in ctrs:
                # shares of the waves' resident time (all three counters count wave quad-cycles)
                wc = med([v["SQ_WAVE_CYCLES"] for _, v in lst])
                if "SQ_WAIT_ANY" in ctrs:
                    wa = med([v["SQ_WAIT_ANY"] for _, v in lst])
                    print(f"  share of resident wave time at a wait (SQ_WAIT_ANY / SQ_WAVE_CYCLES): {wa / wc:.3f}")
                if "SQ_WAIT_INST_ANY" in ctrs:
                    wi = med([v["SQ_WAIT_INST_ANY"] for _, v in lst])
                    print(f"  share of resident wave time waiting to issue (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES): {wi / wc:.3f}")
            if "GRBM_GUI_ACTIVE" in ctrs:
                g = med([v["GRBM_GUI_ACTIVE"] for _, v in lst])
                print(f"  clock GHz (GRBM_GUI_ACTIVE / 8 XCDs / duration): {g / 8 / (ms * 1e6):.2f}")
                if "SQ_VALU_MFMA_BUSY_CYCLES" in ctrs:
                    mb = med([v["SQ_VALU_MFMA_BUSY_CYCLES"] for _, v in lst])
                    print(f"  MFMA busy share at that clock (busy / (1024 SIMDs x cycles)): {mb / (1024 * g / 8):.3f}")
        return 0
    raise SystemExit(f"unknown summary kind {kind!r}")


def run_pmc_probe(n: int) -> int:
    """Short fixed sequence for hardware counters: 4 dense U3 sweeps on
    targets >= 7 of an n-qubit state (k_gate<1, 5, 1, true>), four fused
    5-qubit blocks in each matrix-core mode (one direct, two wide, one
    LDS-staged launch), one six-qubit BF16x3 block, then one plain copy of the
    state (8 * 2^n bytes read, the same written) to scale the counters."""
    import numpy as np
    import torch

    from paper_2511_19291_amd import circuits as C
    from paper_2511_19291_amd import sv

    st = sv.State(n).reset()
    b = C._Builder(n)
    for t in (7, 12, 20, n - 1):
        b.gate("u3", [t], values=[0.3, 1.1, -0.7])
    circ = b.build("pmc_probe")
    st.run(circ)
    torch.cuda.synchronize()
    # fused 5-qubit blocks per matrix-core mode, one per kernel form: lowest
    # target 5 (direct form), >= 6 (wide form, twice), < 5 (LDS-staged form)
    rng = np.random.Generator(np.random.PCG64(7))
    z = rng.normal(size=(32, 32)) + 1j * rng.normal(size=(32, 32))
    q, r = np.linalg.qr(z)
    m = q * (np.diag(r) / np.abs(np.diag(r)))
    blocks = [((9, 8, 7, 6, 5), m), ((n - 1, 20, 14, 10, 6), m), ((11, 10, 9, 8, 7), m), ((n - 1, 12, 3, 2, 0), m)]
    st.apply_fused(blocks, sv.FUSED_FP32_MFMA)
    st.apply_fused(blocks, sv.FUSED_BF16X3)
    # one six-qubit block (BF16x3)
    z6 = rng.normal(size=(64, 64)) + 1j * rng.normal(size=(64, 64))
    q6, r6 = np.linalg.qr(z6)
    st.apply_fused([((n - 1, 20, 14, 10, 7, 6), q6 * (np.diag(r6) / np.abs(np.diag(r6))))], sv.FUSED_BF16X3)
    torch.cuda.synchronize()
    dst = torch.empty_like(st.tensor)
    sv.check(sv.lib().sv_stream_copy(dst.data_ptr(), st.tensor.data_ptr(), 8 * (1 << n),
                                     torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": True, "n": n, "dense_launches": 4, "fused_launches_per_mode": len(blocks),
                      "copy_bytes": 8 * (1 << n),
                      "kernel_source_digest": kernel_source_digest()}), flush=True)
    return 0


def run_adjoint_probe(n: int) -> int:
    """One forward (plain sweeps) and one matrix-core adjoint backward of the
    n-qubit ring of 10 RX/RY layers with CNOT rings, loss <sum Z_i>."""
    import torch

    from paper_2511_19291_amd import circuits as C
    from paper_2511_19291_amd import sv

    circ = C.rxry_ring(n, 10, 5)
    st = sv.State(n).reset().run(circ)
    loss, grad, drift = st.adjoint_grad(circ, C.z_sum_terms(n), block_qubits=sv.ADJOINT_MFMA)
    torch.cuda.synchronize()
    # one plain copy of the state (8 * 2^n bytes each way) to scale byte counters
    dst = torch.empty_like(st.tensor)
    sv.check(sv.lib().sv_stream_copy(dst.data_ptr(), st.tensor.data_ptr(), 8 * (1 << n),
                                     torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    print(json.dumps({"adjoint_probe": True, "n": n, "loss": float(loss[0]), "drift": float(drift[0]),
                      "copy_bytes": 8 * (1 << n)}), flush=True)
    return 0


def run_batch_probe() -> int:
    """The batching workload (256 circuits of 10..20 qubits) in the default
    configuration and with BF16x3 phases, three graph launches each."""
    import torch

    from paper_2511_19291_amd import circuits as C
    from paper_2511_19291_amd import sv

    circs = C.batch_workload(256, 10, 20, 6, 4)
    for cfg in (None, {"phase_mode": 2}):
        plan = sv.BatchPlan(circs, config=cfg)
        dp = plan.pack()
        out = plan.out_buffer()
        for _ in range(3):
            plan.launch(dp, out)
        torch.cuda.synchronize()
        print(json.dumps({"batch_probe": True, "config": plan.info()["config"], "stats": plan.stats()}), flush=True)
        plan.free()
    return 0


if __name__ == "__main__":
    sys.exit(main())
