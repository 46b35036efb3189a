// batch.cpp -- host side of batched execution: validation, the pass planner
// that cuts each large circuit into LDS-tile passes, device tables, and the
// hipGraph that holds the one persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "batch.h"
#include "sv_internal.h"

struct sv_batch_plan_s {
    int n_circ = 0;
    hipStream_t stream = nullptr;
    std::vector<int> n;
    std::vector<int64_t> param_off;
    int64_t n_params_total = 0;
    std::vector<std::vector<sv_op>> ops;       // host copy for the per-gate form
    sv::BCirc* d_circ = nullptr;
    sv::BPass* d_pass = nullptr;
    sv::BOp* d_ops = nullptr;
    sv::BTask* d_tasks = nullptr;
    sv::BPhase* d_phases = nullptr;
    float2* d_arena = nullptr;
    float2* d_mats = nullptr;
    float* d_frag = nullptr;
    int* d_frag_phase = nullptr;
    int n_frag = 0;
    double* d_zpart = nullptr;
    int* d_counter = nullptr;
    int* d_done = nullptr;
    int* d_late = nullptr;                     // per circuit: a wait gave up
    int* d_spin = nullptr;                     // spin limit of the inter-pass waits
    int n_tasks = 0;
    int n_ops = 0;
    int n_pass = 0;
    sv_batch_stats stats{};
    int grid = 1;
    sv_batch_config cfg{};                     // effective configuration
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const double* cap_params = nullptr;
    double* cap_out = nullptr;
    float2* pg_arena = nullptr;                 // per-gate form: one full state per circuit
    std::vector<int64_t> pg_off;
};

namespace sv {

namespace {

void need(bool ok, sv_status st, const std::string& msg)
{
    if (!ok) fail(st, msg);
}

template <class F>
sv_status guarded(F&& f)
{
    try {
        f();
        set_last_error("");
        return SV_OK;
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return SV_ERR_OUT_OF_MEMORY;
    } catch (...) {
        set_last_error("unexpected error");
        return SV_ERR_INVALID_ARGUMENT;
    }
}

uint64_t op_mask(const sv_op& op)
{
    uint64_t m = 0;
    for (int j = 0; j < op.n_targets; ++j) m |= 1ull << op.targets[j];
    for (int j = 0; j < op.n_controls; ++j) m |= 1ull << op.controls[j];
    return m;
}

struct Pass {
    std::vector<int> gates;
    uint64_t tile;
};

// Cut a gate list into passes whose gates all act inside one tile of
// tile_bits qubits that always contains the low qubits. Scanning in order, a
// gate joins the pass when its qubits fit and it touches no qubit of a gate
// already left for a later pass; so gates only move past gates on disjoint
// qubits and the pass sequence equals the circuit.
//
// Qubits 0..run_bits-1 are in every tile, so a tile is made of contiguous
// runs of 2^run_bits amplitudes in the state (the unit of coalesced memory
// access); the rest of the tile (at least five qubits, the most one gate
// touches) is free for the pass's gates. Shorter runs leave more room, so
// fewer passes (fewer round trips of the state through memory).
std::vector<Pass> plan_passes(int n, const std::vector<sv_op>& ops, int tile_bits, int run_bits)
{
    const uint64_t low = (1ull << run_bits) - 1;
    const int room = tile_bits - run_bits;
    std::vector<int> remaining(ops.size());
    std::iota(remaining.begin(), remaining.end(), 0);
    std::vector<Pass> passes;
    while (!remaining.empty()) {
        uint64_t chosen = 0, blocked = 0;
        Pass p;
        std::vector<int> rest;
        for (int g : remaining) {
            const uint64_t gm = op_mask(ops[g]);
            if (gm & blocked) {
                blocked |= gm;
                rest.push_back(g);
                continue;
            }
            const uint64_t hi = gm & ~low;
            if (__builtin_popcountll(chosen | hi) <= room) {
                chosen |= hi;
                p.gates.push_back(g);
            } else {
                blocked |= gm;
                rest.push_back(g);
            }
        }
        uint64_t tile = low | chosen;
        for (int q = 0; q < n && __builtin_popcountll(tile) < tile_bits; ++q) tile |= 1ull << q;
        p.tile = tile;
        passes.push_back(std::move(p));
        remaining.swap(rest);
    }
    return passes;
}

// Cut the gates of one pass (tile-local masks, in pass order) into register
// phases of four qubits, with the same in-order rule as the passes: a gate
// joins the phase when its qubits fit and it touches no qubit of a gate left
// for a later phase. A gate on more than four qubits is a phase of its own
// (run as one LDS sweep, marked by g[0] = -1). Returns the gate order and
// fills the phases (op ranges relative to the pass).
std::vector<int> plan_phases(const std::vector<uint32_t>& masks, int m, std::vector<BPhase>& phases)
{
    std::vector<int> order, remaining(masks.size());
    std::iota(remaining.begin(), remaining.end(), 0);
    while (!remaining.empty()) {
        uint32_t chosen = 0, blocked = 0;
        std::vector<int> take, rest;
        if (__builtin_popcount(masks[remaining[0]]) > kRegBits) {
            take.push_back(remaining[0]);
            rest.assign(remaining.begin() + 1, remaining.end());
            BPhase ph{};
            ph.op_begin = (int)order.size();
            ph.op_end = ph.op_begin + 1;
            ph.g[0] = -1;
            phases.push_back(ph);
            order.push_back(take[0]);
            remaining.swap(rest);
            continue;
        }
        for (int g : remaining) {
            const uint32_t q = masks[g];
            if ((q & blocked) || __builtin_popcount(chosen | q) > kRegBits) {
                blocked |= q;
                rest.push_back(g);
                continue;
            }
            chosen |= q;
            take.push_back(g);
        }
        for (int b = 0; b < m && __builtin_popcount(chosen) < kRegBits; ++b) chosen |= 1u << b;
        BPhase ph{};
        ph.op_begin = (int)order.size();
        ph.op_end = ph.op_begin + (int)take.size();
        for (int b = 0, i = 0; b < m; ++b)
            if ((chosen >> b) & 1) ph.g[i++] = b;
        phases.push_back(ph);
        order.insert(order.end(), take.begin(), take.end());
        remaining.swap(rest);
    }
    return order;
}

template <class T>
T* upload(const std::vector<T>& v)
{
    T* d = nullptr;
    const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
    if (hipMalloc(&d, bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(SV_ERR_OUT_OF_MEMORY, "batch table allocation failed");
    }
    if (!v.empty()) SV_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

void destroy(sv_batch_plan p)
{
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->d_circ);
    (void)hipFree(p->d_pass);
    (void)hipFree(p->d_ops);
    (void)hipFree(p->d_tasks);
    (void)hipFree(p->d_phases);
    (void)hipFree(p->d_arena);
    (void)hipFree(p->d_mats);
    (void)hipFree(p->d_frag);
    (void)hipFree(p->d_frag_phase);
    (void)hipFree(p->d_zpart);
    (void)hipFree(p->d_counter);
    (void)hipFree(p->d_done);
    (void)hipFree(p->d_late);
    (void)hipFree(p->d_spin);
    (void)hipFree(p->pg_arena);
    delete p;
}

sv_batch_config default_config()
{
    sv_batch_config c{};
    c.tile_bits = kMaxTileBits;
    c.threads = 512;
    c.reg_min_bits = 12;
    c.wg_per_cu = 0;
    c.phase_mode = kPhaseFp32;
    c.fuse_min_gates = 3;
    c.run_bits = 3;
    return c;
}

void check_config(const sv_batch_config& c)
{
    need(c.tile_bits >= kMinTileBits && c.tile_bits <= kMaxTileBits, SV_ERR_INVALID_ARGUMENT,
         "tile_bits must be 10..14");
    need(c.threads == 256 || c.threads == 512 || c.threads == 1024, SV_ERR_INVALID_ARGUMENT,
         "threads must be 256, 512 or 1024");
    need(c.reg_min_bits >= kRegBits && c.reg_min_bits <= kMaxTileBits + 1, SV_ERR_INVALID_ARGUMENT,
         "reg_min_bits must be 4..15");
    need(c.wg_per_cu >= 0 && c.wg_per_cu <= 16, SV_ERR_INVALID_ARGUMENT, "wg_per_cu must be 0..16");
    need(c.phase_mode >= kPhaseGates && c.phase_mode <= kPhaseBf16x3, SV_ERR_INVALID_ARGUMENT,
         "phase_mode must be 0 (gates), 1 (FP32 MFMA) or 2 (BF16x3 MFMA)");
    need(c.fuse_min_gates >= 1 && c.fuse_min_gates <= 64, SV_ERR_INVALID_ARGUMENT, "fuse_min_gates must be 1..64");
    need(c.run_bits >= 3 && c.run_bits <= 6 && c.run_bits <= c.tile_bits - 5, SV_ERR_INVALID_ARGUMENT,
         "run_bits must be 3..6 and at most tile_bits - 5");
}

BatchArgs args_of(sv_batch_plan p, const double* params, double* out)
{
    BatchArgs a{};
    a.circ = p->d_circ;
    a.pass = p->d_pass;
    a.ops = p->d_ops;
    a.tasks = p->d_tasks;
    a.phases = p->d_phases;
    a.n_tasks = p->n_tasks;
    a.n_ops = p->n_ops;
    a.n_pass = p->n_pass;
    a.arena = p->d_arena;
    a.mats = p->d_mats;
    a.frag = p->d_frag;
    a.frag_phase = p->d_frag_phase;
    a.n_frag = p->n_frag;
    a.phase_mode = p->cfg.phase_mode;
    a.zpart = p->d_zpart;
    a.params = params;
    a.out = out;
    a.counter = p->d_counter;
    a.done = p->d_done;
    a.late = p->d_late;
    a.spin = p->d_spin;
    a.n_circ = p->n_circ;
    return a;
}

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_batch_default_config(sv_batch_config* out)
{
    return guarded([&] {
        need(out != nullptr, SV_ERR_INVALID_ARGUMENT, "out is NULL");
        *out = default_config();
    });
}

sv_status sv_batch_plan_create_ex(int n_circuits, const int* n_qubits, const sv_op* const* ops, const int* n_ops,
                                  const int* n_params, const sv_batch_config* config, void* stream,
                                  sv_batch_plan* out)
{
    sv_batch_plan p = nullptr;
    const sv_status st = guarded([&] {
        need(out != nullptr, SV_ERR_INVALID_ARGUMENT, "out is NULL");
        *out = nullptr;
        const sv_batch_config cfg = config ? *config : default_config();
        check_config(cfg);
        need(n_circuits >= 1, SV_ERR_INVALID_ARGUMENT, "need at least one circuit");
        need(n_qubits && ops && n_ops && n_params, SV_ERR_INVALID_ARGUMENT, "null array");
        p = new sv_batch_plan_s;
        p->n_circ = n_circuits;
        p->stream = static_cast<hipStream_t>(stream);
        for (int c = 0; c < n_circuits; ++c) {
            const int n = n_qubits[c];
            need(n >= 1 && n <= kBatchMaxQubits, SV_ERR_INVALID_ARGUMENT,
                 "circuit " + std::to_string(c) + ": n_qubits must be 1..24");
            need(n_ops[c] >= 0 && (n_ops[c] == 0 || ops[c]), SV_ERR_INVALID_ARGUMENT, "ops is NULL");
            need(n_params[c] >= 0, SV_ERR_INVALID_ARGUMENT, "negative n_params");
            std::vector<sv_op> v(ops[c], ops[c] + n_ops[c]);
            for (int i = 0; i < n_ops[c]; ++i) {
                const sv_op& op = v[i];
                need(op.kind >= SV_H && op.kind <= SV_RZZ, SV_ERR_UNSUPPORTED,
                     "circuit " + std::to_string(c) + " op " + std::to_string(i) + ": kind not allowed in a batch");
                need(op.n_targets == kind_targets(op.kind), SV_ERR_INVALID_ARGUMENT, "n_targets does not match the kind");
                const sv_status gs = sv_check_gate(n, op.targets, op.n_targets, op.controls, op.n_controls);
                if (gs != SV_OK) fail(gs, "circuit " + std::to_string(c) + " op " + std::to_string(i) + ": " + sv_last_error());
                for (int j = 0; j < kind_nparams(op.kind); ++j)
                    need(op.param[j] >= 0 && op.param[j] < n_params[c], SV_ERR_INVALID_ARGUMENT,
                         "circuit " + std::to_string(c) + " op " + std::to_string(i) + ": parameter index out of range");
            }
            p->n.push_back(n);
            p->param_off.push_back(p->n_params_total);
            p->n_params_total += n_params[c];
            p->ops.push_back(std::move(v));
        }
        // largest circuits first (the atomic queue hands them out in this order)
        std::vector<int> order(n_circuits);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p->n[a] > p->n[b]; });
        std::vector<BCirc> circ;
        std::vector<BPass> pass;
        std::vector<BOp> bops;
        std::vector<BPhase> phase;
        std::vector<int> frag_phase;
        int64_t arena = 0, zrows = 0;
        for (int c : order) {
            const int n = p->n[c];
            const std::vector<sv_op>& v = p->ops[c];
            BCirc bc{};
            bc.n = n;
            bc.m = std::min(n, cfg.tile_bits);
            bc.ntiles = 1 << (n - bc.m);
            bc.out_idx = c;
            bc.arena_off = 0;
            bc.zpart_off = 0;
            if (n > cfg.tile_bits) {
                bc.arena_off = arena;
                arena += 1ll << n;
                bc.zpart_off = zrows;
                zrows += bc.ntiles;
            }
            int32_t circ_fused = 0, circ_gates = 0;   // this circuit's fused phases and one-by-one gates
            std::vector<Pass> pl;
            if (n <= cfg.tile_bits) {
                Pass one;
                one.gates.resize(v.size());
                std::iota(one.gates.begin(), one.gates.end(), 0);
                one.tile = (1ull << n) - 1;
                pl.push_back(std::move(one));
            } else {
                pl = plan_passes(n, v, cfg.tile_bits, cfg.run_bits);
            }
            bc.pass_begin = (int)pass.size();
            for (const Pass& ps : pl) {
                BPass bp{};
                int local[64];
                int j = 0;
                for (int q = 0; q < n; ++q)
                    if ((ps.tile >> q) & 1) {
                        local[q] = j;
                        bp.pos[j++] = q;
                    }
                bp.op_begin = (int)bops.size();
                std::vector<BOp> pops;
                std::vector<uint32_t> masks;
                for (int g : ps.gates) {
                    const sv_op& op = v[g];
                    BOp b{};
                    b.kind = op.kind;
                    b.nt = op.n_targets;
                    b.np = 0;
                    uint32_t mask = 0;
                    for (int t = 0; t < op.n_targets; ++t) {
                        b.pos[b.np++] = local[op.targets[t]];
                        mask |= 1u << local[op.targets[t]];
                    }
                    for (int t = 0; t < op.n_controls; ++t) {
                        b.pos[b.np++] = local[op.controls[t]];
                        b.cmask |= 1u << local[op.controls[t]];
                        mask |= 1u << local[op.controls[t]];
                    }
                    std::sort(b.pos, b.pos + b.np);
                    const int D = 1 << b.nt;
                    for (int r = 0; r < D; ++r) {
                        uint32_t off = 0;
                        for (int t = 0; t < b.nt; ++t)
                            if ((r >> (b.nt - 1 - t)) & 1) off |= 1u << local[op.targets[t]];
                        b.off[r] = off;
                    }
                    for (int t = 0; t < 3; ++t)
                        b.p[t] = t < kind_nparams(op.kind) ? (int)(p->param_off[c] + op.param[t]) : -1;
                    pops.push_back(b);
                    masks.push_back(mask);
                }
                bp.phase_begin = bp.phase_end = (int)phase.size();
                bp.first_frag = -1;
                if (bc.m >= cfg.reg_min_bits) {
                    std::vector<BPhase> ph;
                    const std::vector<int> order = plan_phases(masks, bc.m, ph);
                    for (BPhase& x : ph) {
                        // register positions of each gate's qubits inside the phase
                        for (int oi = x.op_begin; oi < x.op_end && x.g[0] >= 0; ++oi) {
                            BOp& b = pops[order[oi]];
                            auto rpos = [&](int tilebit) {
                                for (int i = 0; i < kRegBits; ++i)
                                    if (x.g[i] == tilebit) return i;
                                return -1;
                            };
                            for (int t = 0; t < b.nt; ++t) b.rt[t] = rpos(__builtin_ctz(b.off[b.nt == 1 ? 1 : (t == 0 ? 2 : 1)]));
                            b.rcmask = 0;
                            for (int q = 0; q < 32; ++q)
                                if ((b.cmask >> q) & 1) b.rcmask |= 1 << rpos(q);
                        }
                        x.op_begin += (int)bops.size();
                        x.op_end += (int)bops.size();
                        // fused on the matrix cores: a phase of enough gates
                        // in a tile of at least 32 units (one wave's product)
                        x.frag = x.next_frag = -1;
                        if (cfg.phase_mode != kPhaseGates && x.g[0] >= 0 && bc.m >= kRegBits + 5 &&
                            x.op_end - x.op_begin >= cfg.fuse_min_gates) {
                            x.frag = (int)frag_phase.size();
                            frag_phase.push_back((int)phase.size());
                        }
                        const int64_t amps = 1ll << n;     // every tile of the pass runs the phase
                        p->stats.n_phases += 1;
                        if (x.frag >= 0) {
                            p->stats.n_fused_phases += 1;
                            p->stats.fused_amp_phases += amps;
                            circ_fused += 1;
                        } else {
                            p->stats.gate_amp_updates += amps * (x.op_end - x.op_begin);
                            circ_gates += x.op_end - x.op_begin;
                        }
                        phase.push_back(x);
                    }
                    bp.phase_end = (int)phase.size();
                    int next = -1;
                    for (int hi = bp.phase_end - 1; hi >= bp.phase_begin; --hi) {
                        phase[hi].next_frag = next;
                        if (phase[hi].frag >= 0) next = phase[hi].frag;
                    }
                    bp.first_frag = next;
                    for (int oi : order) bops.push_back(pops[oi]);
                } else {
                    bops.insert(bops.end(), pops.begin(), pops.end());
                    p->stats.gate_amp_updates += (1ll << n) * (int64_t)pops.size();
                    circ_gates += (int32_t)pops.size();
                }
                bp.op_end = (int)bops.size();
                pass.push_back(bp);
            }
            bc.pass_end = (int)pass.size();
            circ.push_back(bc);
            p->stats.max_circuit_fused_phases = std::max(p->stats.max_circuit_fused_phases, circ_fused);
            p->stats.max_circuit_gate_sweeps = std::max(p->stats.max_circuit_gate_sweeps, circ_gates);
        }
        need(p->n_params_total < (1ll << 31) && bops.size() < (1u << 31) && frag_phase.size() < (1u << 26),
             SV_ERR_UNSUPPORTED, "batch too large");
        // tasks: round r = pass r of every circuit that has one (largest first),
        // all its tiles; the single-task small circuits follow round 0's large ones
        std::vector<BTask> tasks;
        int max_pass = 0;
        for (const BCirc& bc : circ) max_pass = std::max(max_pass, bc.pass_end - bc.pass_begin);
        for (int r = 0; r < max_pass; ++r) {
            for (int ci = 0; ci < (int)circ.size(); ++ci) {
                const BCirc& bc = circ[ci];
                if (bc.ntiles == 1 || r >= bc.pass_end - bc.pass_begin) continue;
                for (int t = 0; t < bc.ntiles; ++t) tasks.push_back(BTask{ci, bc.pass_begin + r, t, 0});
            }
            if (r == 0)
                for (int ci = 0; ci < (int)circ.size(); ++ci)
                    if (circ[ci].ntiles == 1) tasks.push_back(BTask{ci, circ[ci].pass_begin, 0, 0});
        }
        p->n_tasks = (int)tasks.size();
        p->n_ops = (int)bops.size();
        p->n_pass = (int)pass.size();
        p->d_circ = upload(circ);
        p->d_pass = upload(pass);
        p->d_ops = upload(bops);
        p->d_tasks = upload(tasks);
        p->d_phases = upload(phase);
        p->n_frag = (int)frag_phase.size();
        p->d_frag_phase = upload(frag_phase);
        auto dev_alloc = [&](void** ptr, size_t bytes, const char* what) {
            if (hipMalloc(ptr, std::max<size_t>(bytes, 16)) != hipSuccess) {
                (void)hipGetLastError();
                *ptr = nullptr;
                fail(SV_ERR_OUT_OF_MEMORY, std::string("batch ") + what + " allocation failed");
            }
        };
        if (arena > 0) dev_alloc((void**)&p->d_arena, (size_t)arena * sizeof(float2), "state arena");
        dev_alloc((void**)&p->d_mats, (size_t)p->n_ops * kMatStride * sizeof(float2), "matrix table");
        dev_alloc((void**)&p->d_frag, (size_t)p->n_frag * 64 * kFragFloats * sizeof(float), "fragment table");
        dev_alloc((void**)&p->d_zpart, (size_t)zrows * (kBatchMaxQubits + 1) * sizeof(double), "partials");
        dev_alloc((void**)&p->d_done, (size_t)p->n_pass * sizeof(int), "pass counters");
        dev_alloc((void**)&p->d_counter, sizeof(int), "queue counter");
        dev_alloc((void**)&p->d_late, (size_t)n_circuits * sizeof(int), "late flags");
        dev_alloc((void**)&p->d_spin, sizeof(int), "spin limit");
        {
            const int spin = kDefaultSpinLimit;
            SV_HIP(hipMemcpy(p->d_spin, &spin, sizeof(int), hipMemcpyHostToDevice));
        }
        // persistent grid: the requested workgroups per CU, at most as many
        // as are resident at once (LDS, registers), at most one per task
        const int resident = batch_max_wg_per_cu(cfg.threads, cfg.tile_bits, cfg.phase_mode);
        const int per_cu = cfg.wg_per_cu == 0 ? resident : std::min(cfg.wg_per_cu, resident);
        p->cfg = cfg;
        p->cfg.wg_per_cu = per_cu;
        p->grid = std::max(1, std::min(p->n_tasks, device_info().cu_count * per_cu));
        *out = p;
    });
    if (st != SV_OK) destroy(p);
    return st;
}

sv_status sv_batch_plan_create(int n_circuits, const int* n_qubits, const sv_op* const* ops, const int* n_ops,
                               const int* n_params, void* stream, sv_batch_plan* out)
{
    return sv_batch_plan_create_ex(n_circuits, n_qubits, ops, n_ops, n_params, nullptr, stream, out);
}

sv_status sv_batch_plan_info(sv_batch_plan p, sv_batch_config* config, int* grid, int* n_tasks, int* n_passes)
{
    return guarded([&] {
        need(p != nullptr, SV_ERR_INVALID_ARGUMENT, "null plan");
        if (config) *config = p->cfg;
        if (grid) *grid = p->grid;
        if (n_tasks) *n_tasks = p->n_tasks;
        if (n_passes) *n_passes = p->n_pass;
    });
}

sv_status sv_batch_plan_stats(sv_batch_plan p, sv_batch_stats* out)
{
    return guarded([&] {
        need(p != nullptr && out != nullptr, SV_ERR_INVALID_ARGUMENT, "null plan or output");
        *out = p->stats;
        out->n_tasks = p->n_tasks;
        out->n_passes = p->n_pass;
    });
}

sv_status sv_batch_param_layout(sv_batch_plan p, int64_t* param_offsets, int64_t* total)
{
    return guarded([&] {
        need(p != nullptr, SV_ERR_INVALID_ARGUMENT, "null plan");
        if (param_offsets)
            for (int c = 0; c < p->n_circ; ++c) param_offsets[c] = p->param_off[c];
        if (total) *total = p->n_params_total;
    });
}

sv_status sv_batch_launch(sv_batch_plan p, const double* dev_params, double* dev_out)
{
    return guarded([&] {
        need(p != nullptr, SV_ERR_INVALID_ARGUMENT, "null plan");
        need(dev_out != nullptr, SV_ERR_INVALID_ARGUMENT, "dev_out is NULL");
        need(dev_params != nullptr || p->n_params_total == 0, SV_ERR_INVALID_ARGUMENT, "dev_params is NULL");
        const BatchArgs a = args_of(p, dev_params, dev_out);
        if (!p->stream) {
            // the legacy default stream cannot be captured: launch directly
            launch_batch(a, p->grid, p->cfg.threads, p->cfg.tile_bits, p->stream);
            return;
        }
        if (!p->exec || p->cap_params != dev_params || p->cap_out != dev_out) {
            if (p->exec) {
                SV_HIP(hipGraphExecDestroy(p->exec));
                p->exec = nullptr;
            }
            if (p->graph) {
                SV_HIP(hipGraphDestroy(p->graph));
                p->graph = nullptr;
            }
            SV_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
            try {
                launch_batch(a, p->grid, p->cfg.threads, p->cfg.tile_bits, p->stream);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(p->stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            SV_HIP(hipStreamEndCapture(p->stream, &p->graph));
            SV_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
            p->cap_params = dev_params;
            p->cap_out = dev_out;
        }
        SV_HIP(hipGraphLaunch(p->exec, p->stream));
    });
}

sv_status sv_batch_launch_pergate(sv_batch_plan p, const double* dev_params, double* dev_out)
{
    return guarded([&] {
        need(p != nullptr, SV_ERR_INVALID_ARGUMENT, "null plan");
        need(dev_out != nullptr, SV_ERR_INVALID_ARGUMENT, "dev_out is NULL");
        if (!p->pg_arena) {
            int64_t total = 0;
            for (int c = 0; c < p->n_circ; ++c) {
                p->pg_off.push_back(total);
                total += 1ll << p->n[c];
            }
            if (hipMalloc(&p->pg_arena, (size_t)total * sizeof(float2)) != hipSuccess) {
                (void)hipGetLastError();
                p->pg_arena = nullptr;
                fail(SV_ERR_OUT_OF_MEMORY, "per-gate state arena allocation failed");
            }
        }
        std::vector<double> hp((size_t)std::max<int64_t>(p->n_params_total, 1));
        if (p->n_params_total > 0) {
            SV_HIP(hipMemcpyAsync(hp.data(), dev_params, (size_t)p->n_params_total * sizeof(double),
                                  hipMemcpyDeviceToHost, p->stream));
            SV_HIP(hipStreamSynchronize(p->stream));
        }
        std::vector<double> out((size_t)p->n_circ * SV_BATCH_OUT_STRIDE, 0.0);
        for (int c = 0; c < p->n_circ; ++c) {
            const int n = p->n[c];
            sv_state s = nullptr;
            sv_status st = sv_alloc(n, 1, p->pg_arena + p->pg_off[c], p->stream, &s);
            if (st != SV_OK) fail(st, sv_last_error());
            std::vector<double> z(n + 1);
            st = sv_reset(s, 0);
            if (st == SV_OK)
                st = sv_run(s, p->ops[c].data(), (int)p->ops[c].size(), hp.data() + p->param_off[c], 0,
                            (int)(p->n_params_total - p->param_off[c]));
            if (st == SV_OK) st = sv_expval_z_all(s, z.data());
            const std::string err = sv_last_error();
            sv_free(s);
            if (st != SV_OK) fail(st, err);
            for (int i = 0; i < n; ++i) out[(size_t)c * SV_BATCH_OUT_STRIDE + i] = z[i];
        }
        SV_HIP(hipMemcpyAsync(dev_out, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, p->stream));
        SV_HIP(hipStreamSynchronize(p->stream));
    });
}

sv_status sv_batch_set_spin_limit(sv_batch_plan p, int limit)
{
    return guarded([&] {
        need(p != nullptr, SV_ERR_INVALID_ARGUMENT, "null plan");
        if (p->stream) SV_HIP(hipStreamSynchronize(p->stream));
        else SV_HIP(hipDeviceSynchronize());
        SV_HIP(hipMemcpy(p->d_spin, &limit, sizeof(int), hipMemcpyHostToDevice));
    });
}

sv_status sv_batch_plan_free(sv_batch_plan p)
{
    return guarded([&] { destroy(p); });
}

}  // extern "C"
