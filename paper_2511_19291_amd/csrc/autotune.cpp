// autotune.cpp -- measured choice of the launch shapes: the batched launch's
// tile (tile width, threads per workgroup, register phases, workgroups per
// CU, phase fusion and its arithmetic) and the fusion width k and arithmetic
// of a circuit's fused blocks.
// Every candidate is timed on the device with HIP events on the caller's
// stream; candidates whose results disagree with the reference configuration
// are never chosen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "batch.h"
#include "sv_internal.h"

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

void ok_or_throw(sv_status st)
{
    if (st != SV_OK) fail(st, sv_last_error());
}

// Events on one stream; time() returns milliseconds per repetition of f.
struct Timer {
    hipStream_t st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    explicit Timer(hipStream_t s) : st(s)
    {
        SV_HIP(hipEventCreate(&e0));
        SV_HIP(hipEventCreate(&e1));
    }
    ~Timer()
    {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    template <class F>
    double time(int reps, F&& f)
    {
        SV_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) f();
        SV_HIP(hipEventRecord(e1, st));
        SV_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SV_HIP(hipEventElapsedTime(&ms, e0, e1));
        return (double)ms / reps;
    }
};

struct DevBuf {
    void* p = nullptr;
    explicit DevBuf(size_t bytes)
    {
        if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(SV_ERR_OUT_OF_MEMORY, "autotune buffer allocation failed");
        }
    }
    ~DevBuf() { (void)hipFree(p); }
};

// Bound on |d<Z_i>| of one circuit of a plan from its rounding errors.
// Each sweep (a fused 16 x 16 phase, or one gate applied on its own) forms
// every output component as a dot product of L = 2 D real terms whose
// relative errors are bounded by eps: one-by-one FP32 gates (D <= 4)
// (L + 1) u; FP32 phases in the three-real-product form sqrt2 (L + 3) u;
// BF16x3 phases 3 * 2^-16 (split residuals of both operands, the dropped
// lo*lo product) + (3 L + 1) u, with u = 2^-24. Treating the errors as
// independent and mean zero (Hoeffding), a sweep adds about sqrt2 eps to
// ||dpsi||, sweeps add in quadrature, and with a factor 4:
// ||dpsi|| <= B = 4 sqrt(sum 2 eps^2), |d<Z_i>| <= 2 B + B^2.
double batch_z_bound(const sv_batch_stats& s, int phase_mode)
{
    const double u = std::ldexp(1.0, -24);
    const double eps_gate = (8 + 1) * u;
    const double eps_fused = phase_mode == kPhaseBf16x3 ? 3 * std::ldexp(1.0, -16) + (3 * 32 + 1) * u
                                                        : std::sqrt(2.0) * (32 + 3) * u;
    const double var = 2.0 * (s.max_circuit_fused_phases * eps_fused * eps_fused +
                              s.max_circuit_gate_sweeps * eps_gate * eps_gate);
    const double B = 4.0 * std::sqrt(var);
    return 2.0 * B + B * B;
}

bool same_effective(const sv_batch_config& a, const sv_batch_config& b)
{
    auto reg = [](const sv_batch_config& c) { return c.reg_min_bits > c.tile_bits ? 99 : c.reg_min_bits; };
    // without register phases, or with gate-by-gate phases, the fusion threshold is unused
    auto fuse = [&](const sv_batch_config& c) {
        return reg(c) == 99 || c.phase_mode == kPhaseGates ? 0 : c.phase_mode * 100 + c.fuse_min_gates;
    };
    return a.tile_bits == b.tile_bits && a.threads == b.threads && reg(a) == reg(b) && a.wg_per_cu == b.wg_per_cu &&
           fuse(a) == fuse(b) && a.run_bits == b.run_bits;
}

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_batch_autotune(int n_circuits, const int* n_qubits, const sv_op* const* ops, const int* n_ops,
                            const int* n_params, const double* dev_params, int reps, void* stream,
                            sv_batch_config* best, sv_batch_trial* trials, int max_trials, int* n_trials)
{
    return guarded([&] {
        need(best != nullptr, SV_ERR_INVALID_ARGUMENT, "best is NULL");
        need(reps >= 1 && reps <= 1000, SV_ERR_INVALID_ARGUMENT, "reps must be 1..1000");
        need(max_trials >= 0 && (max_trials == 0 || trials), SV_ERR_INVALID_ARGUMENT, "trials is NULL");
        need(n_circuits >= 1, SV_ERR_INVALID_ARGUMENT, "need at least one circuit");
        hipStream_t st = static_cast<hipStream_t>(stream);
        const size_t n_out = (size_t)n_circuits * SV_BATCH_OUT_STRIDE;
        DevBuf dout(n_out * sizeof(double));
        std::vector<double> ref, got(n_out);
        std::vector<sv_batch_trial> done;
        Timer tm(st);
        double ref_bound = -1.0;   // the default configuration's <Z_i> error bound

        auto run = [&](sv_batch_config cfg) -> const sv_batch_trial& {
            for (const sv_batch_trial& t : done)
                if (same_effective(t.config, cfg)) return t;
            sv_batch_plan p = nullptr;
            ok_or_throw(sv_batch_plan_create_ex(n_circuits, n_qubits, ops, n_ops, n_params, &cfg, stream, &p));
            sv_batch_trial t{};
            try {
                ok_or_throw(sv_batch_plan_info(p, &t.config, nullptr, nullptr, nullptr));
                sv_batch_stats stats{};
                ok_or_throw(sv_batch_plan_stats(p, &stats));
                const double bound = batch_z_bound(stats, t.config.phase_mode);
                if (ref_bound < 0.0) ref_bound = bound;
                t.tol = ref_bound + bound;
                double* o = static_cast<double*>(dout.p);
                ok_or_throw(sv_batch_launch(p, dev_params, o));   // warm-up (and graph capture)
                SV_HIP(hipMemcpyAsync(got.data(), o, n_out * sizeof(double), hipMemcpyDeviceToHost, st));
                SV_HIP(hipStreamSynchronize(st));
                t.ms = tm.time(reps, [&] { ok_or_throw(sv_batch_launch(p, dev_params, o)); });
            } catch (...) {
                sv_batch_plan_free(p);
                throw;
            }
            ok_or_throw(sv_batch_plan_free(p));
            if (ref.empty()) ref = got;
            double dev = 0.0;
            for (size_t i = 0; i < n_out; ++i) {
                const double d = std::fabs(got[i] - ref[i]);
                if (std::isnan(d)) {
                    dev = std::numeric_limits<double>::quiet_NaN();   // a timed-out or broken launch
                    break;
                }
                dev = std::max(dev, d);
            }
            t.max_dev = dev;
            // the same effective configuration under another request is not timed again
            for (const sv_batch_trial& u : done)
                if (same_effective(u.config, t.config)) return u;
            done.push_back(t);
            return done.back();
        };
        auto usable = [&](const sv_batch_trial& t) { return t.max_dev <= t.tol; };
        auto better = [&](const sv_batch_trial& a, const sv_batch_trial* b) {
            return usable(a) && (b == nullptr || a.ms < b->ms);
        };

        sv_batch_config base{};
        ok_or_throw(sv_batch_default_config(&base));
        run(base);   // the reference output
        // stage 1: tile width x threads per workgroup
        sv_batch_trial cur = done.front();
        for (int tb = kMinTileBits; tb <= kMaxTileBits; ++tb)
            for (int th : {256, 512, 1024}) {
                sv_batch_config c = base;
                c.tile_bits = tb;
                c.threads = th;
                c.run_bits = std::min(base.run_bits, tb - 5);
                const sv_batch_trial t = run(c);
                if (better(t, &cur)) cur = t;
            }
        // stage 1b: length of the contiguous runs a tile is made of
        for (int rb = 3; rb <= std::min(6, cur.config.tile_bits - 5); ++rb) {
            sv_batch_config c = cur.config;
            c.run_bits = rb;
            const sv_batch_trial t = run(c);
            if (better(t, &cur)) cur = t;
        }
        // stage 2: where register phases start
        for (int rb : {8, 10, 12, 15}) {
            sv_batch_config c = cur.config;
            c.reg_min_bits = rb;
            c.wg_per_cu = 0;
            const sv_batch_trial t = run(c);
            if (better(t, &cur)) cur = t;
        }
        // stage 3: persistent workgroups per CU (fewer than resident)
        for (int w : {1, 2, 4}) {
            sv_batch_config c = cur.config;
            c.wg_per_cu = w;
            const sv_batch_trial t = run(c);
            if (better(t, &cur)) cur = t;
        }
        // stage 4: phase arithmetic (gate by gate, fused on FP32 or BF16x3
        // matrix cores) and the fewest gates a fused phase needs
        for (int pm : {kPhaseGates, kPhaseFp32, kPhaseBf16x3})
            for (int fm : {2, 3, 4, 6}) {
                sv_batch_config c = cur.config;
                c.phase_mode = pm;
                c.fuse_min_gates = fm;
                const sv_batch_trial t = run(c);
                if (better(t, &cur)) cur = t;
            }
        need(usable(cur), SV_ERR_HIP, "no configuration reproduced the reference output");
        *best = cur.config;
        if (n_trials) *n_trials = (int)done.size();
        for (int i = 0; i < (int)done.size() && i < max_trials; ++i) trials[i] = done[i];
    });
}

sv_status sv_fused_autotune(sv_state s, const sv_op* ops, int n_ops, const double* params, int n_params,
                            uint32_t mode_mask, int reps, sv_fusion_choice* best, sv_fusion_choice* trials,
                            int max_trials, int* n_trials)
{
    return guarded([&] {
        need(s != nullptr && s->psi != nullptr, SV_ERR_INVALID_ARGUMENT, "null state");
        need(best != nullptr, SV_ERR_INVALID_ARGUMENT, "best is NULL");
        need(reps >= 1 && reps <= 1000, SV_ERR_INVALID_ARGUMENT, "reps must be 1..1000");
        need(max_trials >= 0 && (max_trials == 0 || trials), SV_ERR_INVALID_ARGUMENT, "trials is NULL");
        need((mode_mask & ~7u) == 0, SV_ERR_INVALID_ARGUMENT, "unknown bits in mode_mask");
        std::vector<sv_fusion_choice> done;
        Timer tm(s->stream);

        // plain per-gate sweeps
        {
            ok_or_throw(sv_run(s, ops, n_ops, params, 0, n_params));
            sv_fusion_choice c{};
            c.max_k = 1;
            c.mode = -1;
            c.n_sweeps = n_ops;
            c.ms = tm.time(reps, [&] { ok_or_throw(sv_run(s, ops, n_ops, params, 0, n_params)); });
            done.push_back(c);
        }
        auto try_fused = [&](int k, int mode) {
            const size_t per = (size_t)2 << (2 * k);
            std::vector<sv_block> blocks(std::max(n_ops, 1));
            std::vector<double> mats(blocks.size() * per);
            int nb = 0;
            const sv_status ps = sv_fuse_plan(s->n, ops, n_ops, params, n_params, k, blocks.data(),
                                              (int)blocks.size(), mats.data(), &nb);
            if (ps == SV_ERR_UNSUPPORTED) return;   // a gate wider than k
            ok_or_throw(ps);
            ok_or_throw(sv_apply_fused(s, blocks.data(), nb, mode));
            sv_fusion_choice c{};
            c.max_k = k;
            c.mode = mode;
            c.n_sweeps = nb;
            c.ms = tm.time(reps, [&] { ok_or_throw(sv_apply_fused(s, blocks.data(), nb, mode)); });
            done.push_back(c);
        };
        if (mode_mask & (1u << SV_FUSED_VALU))
            for (int k = 2; k <= 5; ++k) try_fused(k, SV_FUSED_VALU);
        // the matrix-core forms pad every block of up to five qubits to five,
        // so of those widths the widest plan (fewest sweeps) is the one to time
        if (s->n >= 10) {
            if (mode_mask & (1u << SV_FUSED_FP32_MFMA)) try_fused(5, SV_FUSED_FP32_MFMA);
            if (mode_mask & (1u << SV_FUSED_BF16X3)) try_fused(5, SV_FUSED_BF16X3);
        }
        // six-qubit blocks (BF16x3, off qubits 0..5)
        if (s->n >= 12 && s->n <= 32 && (mode_mask & (1u << SV_FUSED_BF16X3))) try_fused(6, SV_FUSED_BF16X3);
        const sv_fusion_choice* b = &done.front();
        for (const sv_fusion_choice& c : done)
            if (c.ms < b->ms) b = &c;
        *best = *b;
        if (n_trials) *n_trials = (int)done.size();
        for (int i = 0; i < (int)done.size() && i < max_trials; ++i) trials[i] = done[i];
    });
}

}  // extern "C"
