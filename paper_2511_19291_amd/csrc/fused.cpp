// fused.cpp -- host side of the fused-block path: the fusion planner that
// multiplies runs of gates into <= 5-qubit blocks (complex128), and
// sv_apply_fused, which prepares each block's matrix for the MFMA or vector
// kernel and queues one sweep per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <tuple>
#include <vector>

#include "sv_internal.h"

namespace sv {

namespace {

void need(bool ok, sv_status st, const std::string& msg)
{
    if (!ok) fail(st, msg);
}

// ------------------------------------------------------------ blocks

// A block: ordered qubit list (qs[0] = most significant bit of the matrix
// index) and its 2^m x 2^m complex128 matrix, row-major.
struct Blk {
    std::vector<int> qs;
    std::vector<cd> m;
    uint64_t mask = 0;
    int gates = 0;
};

int bitpos(const Blk& b, int q)
{
    const int m = (int)b.qs.size();
    for (int i = 0; i < m; ++i)
        if (b.qs[i] == q) return m - 1 - i;
    return -1;
}

// B <- G B for the gate (M on targets, controls) embedded in the block's
// qubits: applied column by column with the gather / multiply / scatter of
// the gate definition.
void absorb(Blk& b, const cd* M, int k, const int* targets, int nc, const int* controls)
{
    const int m = (int)b.qs.size(), d = 1 << m, D = 1 << k;
    int tp[5], cp[3];
    uint64_t tmask = 0, cmask = 0;
    for (int j = 0; j < k; ++j) { tp[j] = bitpos(b, targets[j]); tmask |= 1ull << tp[j]; }
    for (int j = 0; j < nc; ++j) { cp[j] = bitpos(b, controls[j]); cmask |= 1ull << cp[j]; }
    std::vector<cd> v(D), w(D);
    for (int col = 0; col < d; ++col) {
        for (int base = 0; base < d; ++base) {
            if ((base & tmask) || ((uint64_t)base & cmask) != cmask) continue;
            for (int r = 0; r < D; ++r) {
                int idx = base;
                for (int j = 0; j < k; ++j)
                    if ((r >> (k - 1 - j)) & 1) idx |= 1 << tp[j];
                v[r] = b.m[(size_t)idx * d + col];
            }
            for (int r = 0; r < D; ++r) {
                cd acc = 0.0;
                for (int s = 0; s < D; ++s) acc += M[r * D + s] * v[s];
                w[r] = acc;
            }
            for (int r = 0; r < D; ++r) {
                int idx = base;
                for (int j = 0; j < k; ++j)
                    if ((r >> (k - 1 - j)) & 1) idx |= 1 << tp[j];
                b.m[(size_t)idx * d + col] = w[r];
            }
        }
    }
    b.gates += 1;
}

Blk identity_on(const std::vector<int>& qs)
{
    Blk b;
    b.qs = qs;
    for (int q : qs) b.mask |= 1ull << q;
    const int d = 1 << qs.size();
    b.m.assign((size_t)d * d, 0.0);
    for (int i = 0; i < d; ++i) b.m[(size_t)i * d + i] = 1.0;
    return b;
}

struct PlanGate {
    int k;
    int targets[2];
    int nc;
    int controls[SV_MAX_CONTROLS];
    cd m[16];
    uint64_t mask;
};

// A planned block before its matrix is formed: the qubit list (qs[0] = most
// significant bit of the matrix index) and the circuit's gates in the order
// they are multiplied in.
struct PlanBlock {
    std::vector<int> qs;
    std::vector<int> gates;
    uint64_t mask = 0;
};

// The gate's qubits not yet in the block join it (ascending).
void add_qubits(PlanBlock& b, const PlanGate& g)
{
    uint64_t fresh = g.mask & ~b.mask;
    while (fresh) {
        const int q = __builtin_ctzll(fresh);
        fresh &= fresh - 1;
        b.qs.push_back(q);
        b.mask |= 1ull << q;
    }
}

// Planner A (open blocks). Open blocks hold disjoint qubit sets, so they
// commute and may be closed in any order; a gate joins the open blocks it
// touches (merging them) when the union fits, otherwise the fullest touched
// blocks are closed until it fits. No gate moves past another gate on a
// shared qubit, so the block sequence equals the circuit.
// Widest block allowed on a qubit set: max_k, except that six-qubit blocks
// must keep off qubits 0..5 (the six-qubit matrix-core form streams those as
// its columns); a block touching one of them holds at most five qubits.
int width_limit(uint64_t mask, int max_k) { return max_k == 6 && (mask & 63) ? 5 : max_k; }

std::vector<PlanBlock> plan_open_blocks(const std::vector<PlanGate>& gates, int max_k)
{
    std::vector<PlanBlock> out, open;
    for (int gi = 0; gi < (int)gates.size(); ++gi) {
        const PlanGate& g = gates[gi];
        std::vector<int> hit;
        for (int i = 0; i < (int)open.size(); ++i)
            if (open[i].mask & g.mask) hit.push_back(i);
        auto over = [&](const std::vector<int>& keep) {
            uint64_t u = g.mask;
            for (int i : keep) u |= open[i].mask;
            return __builtin_popcountll(u) > width_limit(u, max_k);
        };
        std::vector<int> keep = hit;
        // close the fullest touched blocks until the gate fits
        while (over(keep)) {
            int best = -1;
            for (int j = 0; j < (int)keep.size(); ++j)
                if (best < 0 || open[keep[j]].qs.size() > open[keep[best]].qs.size()) best = j;
            keep.erase(keep.begin() + best);
        }
        // merge the kept blocks (disjoint qubits: their gates commute) and add the gate
        PlanBlock b;
        for (int i : keep) {
            b.qs.insert(b.qs.end(), open[i].qs.begin(), open[i].qs.end());
            b.gates.insert(b.gates.end(), open[i].gates.begin(), open[i].gates.end());
            b.mask |= open[i].mask;
        }
        add_qubits(b, g);
        b.gates.push_back(gi);
        // closed blocks go out first, in creation order
        std::vector<PlanBlock> next;
        for (int i = 0; i < (int)open.size(); ++i) {
            const bool is_hit = std::find(hit.begin(), hit.end(), i) != hit.end();
            const bool is_kept = std::find(keep.begin(), keep.end(), i) != keep.end();
            if (is_hit && !is_kept) out.push_back(std::move(open[i]));
            else if (!is_hit) next.push_back(std::move(open[i]));
        }
        next.push_back(std::move(b));
        open = std::move(next);
    }
    for (PlanBlock& b : open) out.push_back(std::move(b));
    return out;
}

// Planner B (frontier growth). Blocks are built one at a time from the
// gates whose predecessors (the previous gate on each of their qubits) are
// all placed already: the block repeatedly takes the ready gate that adds
// the fewest new qubits while the block stays within max_k qubits, ties
// broken by `variant` (0: circuit order; 1: most shared qubits, then order;
// 2: lowest qubit, then order). A gate is only ever placed after all its
// predecessors, so the block sequence equals the circuit.
std::vector<PlanBlock> plan_frontier(const std::vector<PlanGate>& gates, int max_k, int variant)
{
    const int G = (int)gates.size();
    std::vector<std::vector<int>> succ(G);
    std::vector<int> indeg(G, 0);
    {
        std::vector<int> last(64, -1);
        for (int i = 0; i < G; ++i) {
            std::vector<int> pred;
            for (int q = 0; q < 64; ++q)
                if ((gates[i].mask >> q) & 1) {
                    if (last[q] >= 0 && std::find(pred.begin(), pred.end(), last[q]) == pred.end()) pred.push_back(last[q]);
                    last[q] = i;
                }
            for (int p : pred) succ[p].push_back(i);
            indeg[i] = (int)pred.size();
        }
    }
    std::vector<int> ready;
    for (int i = 0; i < G; ++i)
        if (indeg[i] == 0) ready.push_back(i);
    std::vector<PlanBlock> out;
    while (!ready.empty()) {
        PlanBlock b;
        for (;;) {
            int best = -1;
            long key0 = 0, key1 = 0, key2 = 0;
            for (int j = 0; j < (int)ready.size(); ++j) {
                const PlanGate& g = gates[ready[j]];
                const uint64_t u = b.mask | g.mask;
                if (__builtin_popcountll(u) > width_limit(u, max_k)) continue;
                const long k0 = __builtin_popcountll(g.mask & ~b.mask);
                long k1 = 0;
                if (variant == 1) k1 = -(long)__builtin_popcountll(g.mask & b.mask);
                else if (variant == 2) k1 = __builtin_ctzll(g.mask);
                const long k2 = ready[j];
                if (best < 0 || std::tie(k0, k1, k2) < std::tie(key0, key1, key2)) {
                    best = j;
                    key0 = k0;
                    key1 = k1;
                    key2 = k2;
                }
            }
            if (best < 0) break;
            const int gi = ready[best];
            ready.erase(ready.begin() + best);
            add_qubits(b, gates[gi]);
            b.gates.push_back(gi);
            for (int s : succ[gi])
                if (--indeg[s] == 0) ready.push_back(s);
        }
        out.push_back(std::move(b));
    }
    return out;
}

// The block's matrix: the product of its gates, in order, over its qubits.
Blk build_block(const PlanBlock& pb, const std::vector<PlanGate>& gates)
{
    Blk b = identity_on(pb.qs);
    for (int gi : pb.gates) {
        const PlanGate& g = gates[gi];
        absorb(b, g.m, g.k, g.targets, g.nc, g.controls);
    }
    return b;
}

// Every planner, the plan with the fewest blocks (ties: the first).
std::vector<PlanBlock> best_plan(const std::vector<PlanGate>& gates, int max_k)
{
    std::vector<PlanBlock> best = plan_open_blocks(gates, max_k);
    for (int v = 0; v < 3; ++v) {
        std::vector<PlanBlock> p = plan_frontier(gates, max_k, v);
        if (p.size() < best.size()) best = std::move(p);
    }
    return best;
}

std::vector<Blk> plan(const std::vector<PlanGate>& gates, int max_k)
{
    const std::vector<PlanBlock> best = best_plan(gates, max_k);
    std::vector<Blk> out;
    out.reserve(best.size());
    for (const PlanBlock& pb : best) out.push_back(build_block(pb, gates));
    return out;
}

}  // namespace

std::vector<GateBlock> plan_gate_blocks(const std::vector<uint64_t>& masks, int max_k)
{
    std::vector<PlanGate> gates(masks.size());
    for (size_t i = 0; i < masks.size(); ++i) {
        // the planners need every gate to fit a block on its own
        need(__builtin_popcountll(masks[i]) <= max_k, SV_ERR_UNSUPPORTED, "a gate has more qubits than the block width");
        gates[i].mask = masks[i];
    }
    std::vector<GateBlock> out;
    for (PlanBlock& b : best_plan(gates, max_k)) out.push_back(GateBlock{std::move(b.qs), std::move(b.gates)});
    return out;
}

namespace {

uint16_t bf16_rne_bits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    const uint32_t lsb = (u >> 16) & 1;
    u += 0x7fff + lsb;
    return (uint16_t)(u >> 16);
}

float bf16_round(float x)
{
    const uint32_t u = (uint32_t)bf16_rne_bits(x) << 16;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

void ensure_fused(sv_state s, size_t bytes)
{
    if (bytes <= s->dfused_cap) return;
    if (s->dfused) {
        SV_HIP(hipStreamSynchronize(s->stream));
        SV_HIP(hipFree(s->dfused));
        s->dfused = nullptr;
        s->dfused_cap = 0;
    }
    if (hipMalloc(&s->dfused, bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(SV_ERR_OUT_OF_MEMORY, "fused matrix buffer allocation failed");
    }
    s->dfused_cap = bytes;
}

}  // namespace


}  // namespace sv

using namespace sv;

extern "C" sv_status sv_fuse_plan(int n_qubits, const sv_op* ops, int n_ops, const double* params, int n_params,
                                  int max_k, sv_block* out_blocks, int max_blocks, double* out_matrices,
                                  int* n_blocks_out)
{
    try {
        need(n_qubits >= 1 && n_qubits <= SV_MAX_QUBITS, SV_ERR_INVALID_ARGUMENT, "n_qubits must be in [1, 34]");
        need(max_k >= 1 && max_k <= SV_MAX_FUSED_TARGETS, SV_ERR_INVALID_ARGUMENT, "max_k must be 1..6");
        need(n_ops >= 0 && (n_ops == 0 || ops), SV_ERR_INVALID_ARGUMENT, "ops is NULL");
        need(out_blocks && out_matrices && n_blocks_out, SV_ERR_INVALID_ARGUMENT, "output pointer is NULL");
        std::vector<PlanGate> gates;
        for (int i = 0; i < n_ops; ++i) {
            const sv_op& op = ops[i];
            PlanGate g{};
            int k = 0;
            need(op.n_controls >= 0 && op.n_controls <= SV_MAX_CONTROLS, SV_ERR_UNSUPPORTED, "at most 3 controls");
            need(sv_check_gate(n_qubits, op.targets, op.n_targets, op.controls, op.n_controls) == SV_OK,
                 SV_ERR_QUBIT_OUT_OF_RANGE, std::string("bad gate ") + std::to_string(i) + ": " + sv_last_error());
            for (int j = 0; j < 3; ++j)
                if (op.param[j] >= 0) need(op.param[j] < n_params && params, SV_ERR_INVALID_ARGUMENT, "param index out of range");
            gate_matrix_of_op(op, params, g.m, &k);
            need(k == op.n_targets, SV_ERR_INVALID_ARGUMENT, "n_targets does not match the gate kind");
            g.k = k;
            g.nc = op.n_controls;
            g.mask = 0;
            for (int j = 0; j < k; ++j) { g.targets[j] = op.targets[j]; g.mask |= 1ull << op.targets[j]; }
            for (int j = 0; j < g.nc; ++j) { g.controls[j] = op.controls[j]; g.mask |= 1ull << op.controls[j]; }
            need(__builtin_popcountll(g.mask) <= max_k, SV_ERR_UNSUPPORTED, "a gate has more qubits than max_k");
            gates.push_back(g);
        }
        std::vector<Blk> blocks = plan(gates, max_k);
        need((int)blocks.size() <= max_blocks, SV_ERR_INVALID_ARGUMENT, "max_blocks too small");
        const size_t stride = (size_t)2 * (1u << max_k) * (1u << max_k);
        for (size_t bi = 0; bi < blocks.size(); ++bi) {
            const Blk& b = blocks[bi];
            sv_block& o = out_blocks[bi];
            o.k = (int)b.qs.size();
            for (int j = 0; j < SV_MAX_FUSED_TARGETS; ++j) o.targets[j] = j < o.k ? b.qs[j] : -1;
            double* dst = out_matrices + bi * stride;
            for (size_t i = 0; i < b.m.size(); ++i) {
                dst[2 * i] = b.m[i].real();
                dst[2 * i + 1] = b.m[i].imag();
            }
            o.matrix = dst;
        }
        *n_blocks_out = (int)blocks.size();
        return SV_OK;
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.st;
    } catch (...) {
        return SV_ERR_INVALID_ARGUMENT;
    }
}

namespace {

// sv_apply_fused and sv_apply_fused_rows: with per_row, each block's matrix
// holds one 2^k x 2^k matrix per batch row (row r at matrix + r 2 4^k
// doubles), and each row's sweep reads its own.
sv_status apply_fused_impl(sv_state s, const sv_block* blocks, int n_blocks, int mode, bool per_row)
{
    try {
        need(s != nullptr && s->psi != nullptr, SV_ERR_INVALID_ARGUMENT, "null state");
        need(mode == SV_FUSED_FP32_MFMA || mode == SV_FUSED_BF16X3 || mode == SV_FUSED_VALU,
             SV_ERR_INVALID_ARGUMENT, "unknown fused mode");
        need(n_blocks >= 0 && (n_blocks == 0 || blocks), SV_ERR_INVALID_ARGUMENT, "blocks is NULL");
        const bool mfma = mode != SV_FUSED_VALU;
        if (per_row) need(mfma, SV_ERR_UNSUPPORTED, "per-row matrices run in the MFMA modes only");
        const int nmat = per_row ? s->batch : 1;
        for (int i = 0; i < n_blocks; ++i) {
            const sv_block& b = blocks[i];
            need(b.k >= 1 && b.k <= SV_MAX_FUSED_TARGETS, SV_ERR_INVALID_ARGUMENT, "block k must be 1..6");
            need(b.matrix != nullptr, SV_ERR_INVALID_ARGUMENT, "block matrix is NULL");
            uint64_t seen = 0;
            for (int j = 0; j < b.k; ++j) {
                need(b.targets[j] >= 0 && b.targets[j] < s->n, SV_ERR_QUBIT_OUT_OF_RANGE, "block target out of range");
                need(!((seen >> b.targets[j]) & 1), SV_ERR_QUBIT_OVERLAP, "block target used twice");
                seen |= 1ull << b.targets[j];
            }
            if (mfma) need(s->n >= 10, SV_ERR_INVALID_ARGUMENT, "the MFMA fused modes need n >= 10");
            if (b.k == 6) {
                need(!per_row, SV_ERR_UNSUPPORTED, "per-row matrices take blocks of at most five qubits");
                need(mode == SV_FUSED_BF16X3, SV_ERR_UNSUPPORTED, "six-qubit blocks run in the BF16X3 mode only");
                need((seen & 63) == 0, SV_ERR_UNSUPPORTED, "six-qubit blocks need every target >= 6");
                need(s->n >= 12 && s->n <= 32, SV_ERR_UNSUPPORTED, "six-qubit blocks need 12 <= n <= 32");
            }
        }
        if (n_blocks == 0) return SV_OK;
        // per-block device payload (16-byte multiples)
        const size_t per5 = mfma ? (size_t)3 * 64 * 64 * sizeof(float)
                                 : (size_t)32 * 32 * sizeof(float2) + 32 * sizeof(uint64_t) + 8 * sizeof(int);
        std::vector<size_t> off(n_blocks + 1, 0);
        for (int i = 0; i < n_blocks; ++i)
            off[i + 1] = off[i] + (size_t)nmat * (((blocks[i].k == 6 ? fused6_matrix_bytes() : per5) + 15) / 16 * 16);
        std::vector<unsigned char> host(off[n_blocks], 0);
        std::vector<std::array<int, 6>> tgt(n_blocks);
        for (int i = 0; i < n_blocks; ++i) {
            const sv_block& b = blocks[i];
            const int k = b.k, D = 1 << k;
            unsigned char* dst = host.data() + off[i];
            if (k == 6) {
                // real 128 x 128 embedding, split into BF16 hi and lo parts
                std::vector<float> hi(128 * 128), lo(128 * 128);
                for (int r = 0; r < 64; ++r)
                    for (int c = 0; c < 64; ++c) {
                        const double* e = b.matrix + 2 * ((size_t)r * 64 + c);
                        const float re = (float)e[0], im = (float)e[1];
                        const float v[4] = {re, -im, im, re};
                        const int at[4] = {r * 128 + c, r * 128 + 64 + c, (64 + r) * 128 + c, (64 + r) * 128 + 64 + c};
                        for (int q = 0; q < 4; ++q) {
                            hi[at[q]] = bf16_round(v[q]);
                            lo[at[q]] = bf16_round(v[q] - hi[at[q]]);
                        }
                    }
                fused6_layout(hi.data(), lo.data(), reinterpret_cast<uint16_t*>(dst));
                for (int j = 0; j < 6; ++j) tgt[i][j] = b.targets[j];
            } else if (mfma) {
                // pad to five targets with identity qubits (lowest free qubits,
                // appended as the least significant bits of the matrix index)
                int t5[5], kk = k;
                uint64_t used = 0;
                for (int j = 0; j < k; ++j) { t5[j] = b.targets[j]; used |= 1ull << b.targets[j]; }
                for (int q = 0; q < s->n && kk < 5; ++q)
                    if (!((used >> q) & 1)) { t5[kk++] = q; used |= 1ull << q; }
                const int pad = 5 - k;
                for (int j = 0; j < 5; ++j) tgt[i][j] = t5[j];
                for (int mi = 0; mi < nmat; ++mi) {
                    const double* bm = b.matrix + (size_t)mi * 2 * D * D;
                    float* A = reinterpret_cast<float*>(dst + (size_t)mi * per5);
                    for (int r = 0; r < 32; ++r)
                        for (int c = 0; c < 32; ++c) {
                            // M5 = M (x) I_{2^pad}
                            cd v = 0.0;
                            if ((r & ((1 << pad) - 1)) == (c & ((1 << pad) - 1))) {
                                const double* e = bm + 2 * ((size_t)(r >> pad) * D + (c >> pad));
                                v = cd(e[0], e[1]);
                            }
                            const float re = (float)v.real(), im = (float)v.imag();
                            A[r * 64 + c] = re;
                            A[r * 64 + 32 + c] = -im;
                            A[(32 + r) * 64 + c] = im;
                            A[(32 + r) * 64 + 32 + c] = re;
                        }
                    // the FP32 products' left operands in fragment order: element
                    // (b, q, lane, e) = A~[32 b + lane % 32][2 (4 q + e) + lane / 32]
                    float* F = A + 2 * 64 * 64;
                    for (int b = 0; b < 2; ++b)
                        for (int q = 0; q < 8; ++q)
                            for (int l = 0; l < 64; ++l)
                                for (int e = 0; e < 4; ++e)
                                    F[((b * 8 + q) * 64 + l) * 4 + e] =
                                        A[(32 * b + (l & 31)) * 64 + 2 * (4 * q + e) + (l >> 5)];
                    if (mode == SV_FUSED_BF16X3) {
                        float* L = A + 64 * 64;
                        for (int q = 0; q < 64 * 64; ++q) {
                            const float hi = bf16_round(A[q]);
                            L[q] = A[q] - hi;
                            A[q] = hi;
                        }
                        // the BF16 products' left operands in fragment order (in place
                        // of the FP32 fragments): the 8 values of (b, s, part, lane) =
                        // part [32 b + lane % 32][16 s + 8 (lane / 32) + q], part 0 the
                        // hi values, 1 the lo values rounded to BF16
                        uint16_t* H = reinterpret_cast<uint16_t*>(F);
                        for (int b = 0; b < 2; ++b)
                            for (int st = 0; st < 4; ++st)
                                for (int part = 0; part < 2; ++part)
                                    for (int l = 0; l < 64; ++l)
                                        for (int q = 0; q < 8; ++q) {
                                            const int at = (32 * b + (l & 31)) * 64 + 16 * st + 8 * (l >> 5) + q;
                                            H[((((b * 4 + st) * 2 + part) * 64) + l) * 8 + q] =
                                                bf16_rne_bits(part == 0 ? A[at] : L[at]);
                                        }
                    }
                }
            } else {
                float2* m = reinterpret_cast<float2*>(dst);
                for (int q = 0; q < D * D; ++q)
                    m[q] = make_float2((float)b.matrix[2 * q], (float)b.matrix[2 * q + 1]);
                uint64_t* moff = reinterpret_cast<uint64_t*>(dst + 32 * 32 * sizeof(float2));
                for (int r = 0; r < D; ++r) {
                    uint64_t off = 0;
                    for (int j = 0; j < k; ++j)
                        if ((r >> (k - 1 - j)) & 1) off |= 1ull << b.targets[j];
                    moff[r] = off;
                }
                int* pos = reinterpret_cast<int*>(dst + 32 * 32 * sizeof(float2) + 32 * sizeof(uint64_t));
                for (int j = 0; j < k; ++j) pos[j] = b.targets[j];
                std::sort(pos, pos + k);
            }
        }
        ensure_fused(s, host.size());
        // pageable source: the copy has consumed `host` when the call returns
        SV_HIP(hipMemcpyAsync(s->dfused, host.data(), host.size(), hipMemcpyHostToDevice, s->stream));
        unsigned char* dev = static_cast<unsigned char*>(s->dfused);
        for (int i = 0; i < n_blocks; ++i) {
            unsigned char* p = dev + off[i];
            if (blocks[i].k == 6) {
                Fused6Launch f{};
                f.psi = s->psi;
                f.N = s->N;
                f.nrows = s->batch;
                for (int j = 0; j < 6; ++j) f.targets[j] = tgt[i][j];
                f.amat = reinterpret_cast<const uint16_t*>(p);
                launch_fused_wide6(f, s->stream);
            } else if (mfma) {
                FusedLaunch f{};
                f.psi = s->psi;
                f.N = s->N;
                f.nrows = s->batch;
                for (int j = 0; j < 5; ++j) f.targets[j] = tgt[i][j];
                f.mode = mode;
                f.amat = reinterpret_cast<const float*>(p);
                f.amat_stride = per_row ? (uint32_t)(per5 / sizeof(float)) : 0u;
                launch_fused_mfma(f, s->stream);
            } else {
                FusedValuLaunch f{};
                f.psi = s->psi;
                f.N = s->N;
                f.nrows = s->batch;
                f.k = blocks[i].k;
                f.m = reinterpret_cast<const float2*>(p);
                f.moff = reinterpret_cast<const uint64_t*>(p + 32 * 32 * sizeof(float2));
                f.pos = reinterpret_cast<const int*>(p + 32 * 32 * sizeof(float2) + 32 * sizeof(uint64_t));
                launch_fused_valu(f, s->stream);
            }
        }
        return SV_OK;
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.st;
    } catch (...) {
        return SV_ERR_INVALID_ARGUMENT;
    }
}

}  // namespace

extern "C" sv_status sv_apply_fused(sv_state s, const sv_block* blocks, int n_blocks, int mode)
{
    return apply_fused_impl(s, blocks, n_blocks, mode, false);
}

extern "C" sv_status sv_apply_fused_rows(sv_state s, const sv_block* blocks, int n_blocks, int mode)
{
    return apply_fused_impl(s, blocks, n_blocks, mode, true);
}
