// batch.h -- device tables of a batch plan (shared by batch.cpp and
// k_batch.hip; not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sv {

constexpr int kMaxTileBits = 14;      // widest LDS tile: 2^14 complex64 = 128 KiB
constexpr int kMinTileBits = 10;
constexpr int kBatchMaxQubits = 24;
constexpr int kMatStride = 16;        // complex64 entries reserved per gate matrix

constexpr int kRegBits = 4;           // register blocking: 16 amplitudes per unit

// One gate with tile-local qubit positions and its precomputed addressing.
struct BOp {
    int kind;
    int nt;                           // 1 or 2 targets
    int np;                           // number of positions where zeros are inserted
    int pos[5];                       // tile-local targets and controls, ascending
    uint32_t cmask;                   // tile-local control bits
    uint32_t off[4];                  // member offsets (target bits by member index)
    int p[3];                         // absolute parameter indices in the launch's block, -1 = none
    int rt[2];                        // register phase: target bits within the phase's 4 qubits
    int rcmask;                       // register phase: control bits within the phase's 4 qubits
};

// A register phase: gates [op_begin, op_end) all act inside the four
// tile-local qubits g[0..3] (ascending); each thread holds the 16 amplitudes
// that differ only in those qubits and applies the gates in registers. A
// fused phase (frag >= 0) instead applies the product of its gates, one
// 16 x 16 unitary, on the matrix cores; its operand fragments are entry
// `frag` of the fragment table.
struct BPhase {
    int op_begin;
    int op_end;
    int g[kRegBits];
    int frag;                         // -1: gate by gate in registers
    int next_frag;                    // fragment of the next fused phase of the pass, -1 = none
};

// Phase arithmetic (sv_batch_config.phase_mode).
constexpr int kPhaseGates = 0;        // every gate applied on its own
constexpr int kPhaseFp32 = 1;         // fused phases on FP32 MFMA
constexpr int kPhaseBf16x3 = 2;       // fused phases as BF16 x3 products, FP32 accumulation
constexpr int kFragFloats = 16;       // per lane and fused phase: 64 bytes (16 FP32 or 32 BF16)

// A pass: gates [op_begin, op_end) all act inside the tile whose bit j is
// qubit pos[j] (ascending). When phase_begin < phase_end the gates run as
// those register phases instead of one LDS sweep each.
struct BPass {
    int op_begin;
    int op_end;
    int phase_begin;
    int phase_end;
    int first_frag;                   // fragment of the pass's first fused phase, -1 = none
    int pos[kMaxTileBits];
};

struct BCirc {
    int n;
    int m;                            // tile bits: min(n, the plan's tile width)
    int pass_begin;
    int pass_end;
    int64_t arena_off;                // amplitude offset of the state in the arena (n > m)
    int64_t zpart_off;                // first row of this circuit's per-tile <Z> partials
    int ntiles;                       // 2^(n - m)
    int out_idx;                      // row of the output
};

// A unit of work: one tile of one pass of one circuit. Tasks are ordered so
// that every tile of a pass precedes every tile of the next pass of the same
// circuit: a task only ever waits for tasks handed out before it.
struct BTask {
    int circ;
    int pass;
    int tile;
    int pad;
};

struct BatchArgs {
    const BCirc* circ;
    const BPass* pass;
    const BOp* ops;
    const BTask* tasks;
    const BPhase* phases;
    int n_tasks;
    int n_ops;
    int n_pass;
    float2* arena;
    float2* mats;                     // n_ops * kMatStride complex64
    float* frag;                      // n_frag * 64 lanes * kFragFloats: fused-phase operands
    const int* frag_phase;            // phase of each fragment
    int n_frag;
    int phase_mode;
    double* zpart;                    // per-tile partials [row][kBatchMaxQubits + 1]
    const double* params;
    double* out;
    int* counter;                     // next task
    int* done;                        // finished tiles per pass
    int* late;                        // per circuit: 1 once any tile gave up waiting for its previous pass
    const int* spin;                  // polls before an inter-pass wait gives up (< 0: give up at once)
    int n_circ;
};

// polls of the bounded inter-pass wait before it gives up (each poll sleeps
// ~4 x 64 cycles): far beyond any real wait, short of a hang
constexpr int kDefaultSpinLimit = 1 << 24;

// dynamic LDS of one workgroup for tiles of 2^tile_bits amplitudes
size_t batch_lds_bytes(int tile_bits);
// resident workgroups per CU of the persistent kernel (also raises the
// kernel's dynamic-LDS limit to that size)
int batch_max_wg_per_cu(int threads, int tile_bits, int phase_mode);
void launch_batch(const BatchArgs& a, int grid, int threads, int tile_bits, hipStream_t st);

}  // namespace sv
