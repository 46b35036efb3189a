// batch.h -- device tables of a batch plan (shared by batch.cpp and
// k_batch.hip; not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sv {

constexpr int kTileBits = 14;         // LDS tile: 2^14 complex64 = 128 KiB
constexpr int kLowBits = 6;           // qubits 0..5 are in every tile (runs of 64 amplitudes)
constexpr int kBatchMaxQubits = 24;

// One gate with tile-local qubit positions.
struct BOp {
    int kind;
    int nt;
    int nc;
    int t[2];
    int c[3];
    int p[3];                         // parameter indices in the circuit's row, -1 = none
    int pad;
};

// A pass: gates [op_begin, op_end) all act inside the tile whose bit j is
// qubit pos[j] (ascending).
struct BPass {
    int op_begin;
    int op_end;
    int pos[kTileBits];
};

struct BCirc {
    int n;
    int m;                            // tile bits: min(n, kTileBits)
    int pass_begin;
    int pass_end;
    int64_t param_off;                // first parameter in the launch's parameter block
    int64_t arena_off;                // amplitude offset of the state in the arena (n > kTileBits)
    int out_idx;                      // row of the output
    int pad;
};

struct BatchArgs {
    const BCirc* circ;
    const BPass* pass;
    const BOp* ops;
    float2* arena;
    const double* params;
    double* out;
    int* counter;
    int n_circ;
};

void launch_batch(const BatchArgs& a, int grid, hipStream_t st);

}  // namespace sv
