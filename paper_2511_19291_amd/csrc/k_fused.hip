// k_fused.hip -- one fused k-qubit gate block per sweep on the matrix cores.
//
// A block is (M, T): a 32 x 32 complex matrix on five ordered target qubits
// (Alg. 1 of Sec. 4.1.1 with |Q| = 5; smaller blocks are padded with identity
// qubits on the host). Viewing the state as X[r][j] with r the five target
// bits (T[0] most significant) and j every other bit, the block computes
// Y = M X over all 2^(n-5) columns -- a dense contraction.
//
// Tiling: a tile is 32 rows x 32 columns = 1024 amplitudes, the columns being
// the five lowest non-target qubits. The tile's ten bit positions therefore
// include every bit below the fifth-lowest non-target, so its memory image is
// made of contiguous runs of at least 32 amplitudes (256 bytes). Each wave
// owns one tile at a time:
//   1. coalesced float4 loads in memory order -> LDS, split into real and
//      imaginary planes;
//   2. complex product on MFMA as a real 64 x 64 product
//      [Yr; Yi] = [[Mr, -Mi], [Mi, Mr]] [Xr; Xi]:
//      FP32: v_mfma_f32_32x32x2_f32, 2 x 32 k-steps;
//      BF16X3: x = x_hi + x_lo with both parts rounded to BF16 (RNE), products
//      hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16, FP32 accumulation;
//      the left operand (the block matrix) stays in registers for the whole
//      sweep;
//   3. results -> LDS -> coalesced float4 stores in memory order.
#include <cstring>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 1;
constexpr int kXs = 33;              // FP32 layout Xs[64][33]: [k][col]
constexpr int kXt = 68;              // BF16 layout Xt[32][68]: [col][k]
constexpr int kWaveLds = 64 * kXs > 32 * kXt ? 64 * kXs : 32 * kXt;   // floats per wave

struct KFused {
    float2* psi;
    uint64_t N;
    uint64_t n_tiles;          // per row
    int pos[10];               // tile bit positions, ascending
    uint64_t bit_off64[10];    // amplitude offset of tile bit b (= 1 << pos[b])
    int bit_row[10];           // row-index contribution of tile bit b (0 if a column bit)
    int bit_col[10];           // column-index contribution of tile bit b (0 if a row bit)
    const float* amat;         // FP32: A~[64][64]; BF16X3: hi A~[64][64] then lo A~[64][64] (as float)
    uint32_t amat_stride;      // floats between batch rows' matrices (0: one matrix for every row)
};

__device__ __forceinline__ bf16x8 to_bf16(const float (&x)[8])
{
    bf16x8 r;
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = (__bf16)x[q];
    return r;
}

// MODE 0: FP32 MFMA; MODE 1: BF16 x3.
template <int MODE>
__global__ __launch_bounds__(kWaves * 64) void k_fused(KFused a)
{
    __shared__ float lds[kWaves * kWaveLds];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    float* xs = lds + wave * kWaveLds;
    float2* psi = a.psi + (uint64_t)blockIdx.y * a.N;
    const float* am = a.amat + (size_t)blockIdx.y * a.amat_stride;      // this row's matrix
    const int h = lane >> 5, c32 = lane & 31;

    // per-lane part of the tile index L = 2*lane + 128*i (+ e): bits 1..6
    uint64_t lane_off = 0;
    int lane_r = 0, lane_c = 0;
#pragma unroll
    for (int b = 1; b <= 6; ++b)
        if ((lane >> (b - 1)) & 1) {
            lane_off += a.bit_off64[b];
            lane_r += a.bit_row[b];
            lane_c += a.bit_col[b];
        }
    uint64_t i_off[8];
    int i_r[8], i_c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        i_off[i] = 0;
        i_r[i] = 0;
        i_c[i] = 0;
#pragma unroll
        for (int b = 7; b <= 9; ++b)
            if ((i >> (b - 7)) & 1) {
                i_off[i] += a.bit_off64[b];
                i_r[i] += a.bit_row[b];
                i_c[i] += a.bit_col[b];
            }
    }
    const int r0 = a.bit_row[0], c0 = a.bit_col[0];   // bit 0 of L (the second amplitude of a float4)

    // left operand fragments, loaded once
    float afr[2][32];
    bf16x8 ahi[2][4], alo[2][4];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                // fragment-ordered copy after the two 64 x 64 parts:
                // element (b, q, lane, e) = A~[32 b + lane % 32][2 (4 q + e) + lane / 32]
                const float4 t4 = reinterpret_cast<const float4*>(am + 2 * 64 * 64)[(b * 8 + q) * 64 + lane];
                afr[b][4 * q] = t4.x;
                afr[b][4 * q + 1] = t4.y;
                afr[b][4 * q + 2] = t4.z;
                afr[b][4 * q + 3] = t4.w;
            }
    } else {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                // fragment-ordered BF16 copy after the two 64 x 64 parts: the 8
                // values of (b, s, part, lane) = part [32 b + lane % 32][16 s + 8 (lane / 32) + q]
                const u32x4* fb = reinterpret_cast<const u32x4*>(am + 2 * 64 * 64);
                ahi[b][s] = __builtin_bit_cast(bf16x8, fb[((b * 4 + s) * 2 + 0) * 64 + lane]);
                alo[b][s] = __builtin_bit_cast(bf16x8, fb[((b * 4 + s) * 2 + 1) * 64 + lane]);
            }
    }

    const uint64_t waves_total = (uint64_t)gridDim.x * kWaves;
    const uint64_t iters = (a.n_tiles + waves_total - 1) / waves_total;
    for (uint64_t it = 0; it < iters; ++it) {
        const uint64_t tile = it * waves_total + (uint64_t)blockIdx.x * kWaves + wave;
        const bool live = tile < a.n_tiles;
        const uint64_t base = insert_zeros(live ? tile : 0, a.pos, 10);
        // 1. load the tile in memory order, scatter into LDS planes
        float4 v[8];
        if (live) {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = ld4(psi + base + lane_off + i_off[i]);
        }
        __syncthreads();   // previous tile's results have been read from LDS
        if (live) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int r = lane_r + i_r[i], c = lane_c + i_c[i];
                if constexpr (MODE == 0) {
                    xs[r * kXs + c] = v[i].x;
                    xs[(32 + r) * kXs + c] = v[i].y;
                    xs[(r + r0) * kXs + c + c0] = v[i].z;
                    xs[(32 + r + r0) * kXs + c + c0] = v[i].w;
                } else {
                    xs[c * kXt + r] = v[i].x;
                    xs[c * kXt + 32 + r] = v[i].y;
                    xs[(c + c0) * kXt + r + r0] = v[i].z;
                    xs[(c + c0) * kXt + 32 + r + r0] = v[i].w;
                }
            }
        }
        __syncthreads();
        // 2. products on the matrix cores
        f32x16 acc0 = {0}, acc1 = {0};
        if (live) {
            if constexpr (MODE == 0) {
#pragma unroll
                for (int s = 0; s < 32; ++s) {
                    const float bv = xs[(2 * s + h) * kXs + c32];
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[0][s], bv, acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[1][s], bv, acc1, 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const float4 p0 = *reinterpret_cast<const float4*>(xs + c32 * kXt + 16 * s + 8 * h);
                    const float4 p1 = *reinterpret_cast<const float4*>(xs + c32 * kXt + 16 * s + 8 * h + 4);
                    float xh[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w}, xl[8];
                    const bf16x8 bh = to_bf16(xh);
#pragma unroll
                    for (int q = 0; q < 8; ++q) xl[q] = xh[q] - (float)bh[q];
                    const bf16x8 bl = to_bf16(xl);
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        f32x16& acc = b == 0 ? acc0 : acc1;
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[b][s], bh, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[b][s], bl, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[b][s], bh, acc, 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();   // every lane has read its B operands
        // 3. results to LDS as Ys[64][33] (rows 0..31 real, 32..63 imaginary)
        if (live) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int row = 8 * (q >> 2) + 4 * h + (q & 3);
                xs[row * kXs + c32] = acc0[q];
                xs[(32 + row) * kXs + c32] = acc1[q];
            }
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int r = lane_r + i_r[i], c = lane_c + i_c[i];
                float4 o;
                o.x = xs[r * kXs + c];
                o.y = xs[(32 + r) * kXs + c];
                o.z = xs[(r + r0) * kXs + c + c0];
                o.w = xs[(32 + r + r0) * kXs + c + c0];
                st4(psi + base + lane_off + i_off[i], o);
            }
        }
    }
}

// Direct form for blocks whose five targets are all >= 5 (then the columns are
// qubits 0..4, so every row of a tile is 32 consecutive amplitudes, 256 B):
// each lane loads the matrix-core operands straight from memory and stores
// its accumulators straight back -- no LDS staging. Lane (h, c) of the
// 32x32x2 FP32 operand layout needs X~[2s + h][c]: amplitude (row 2s + h,
// column c) gives the real part for k-step s and the imaginary part for
// k-step s + 16. For the 32x32x16 BF16 layout lane (h, c) needs rows
// 8h + q and 16 + 8h + q (q < 8). Accumulator q of lane (h, c) is output row
// 8 (q / 4) + 4 h + q % 4, column c. Offsets fit 32 bits (n <= 32).
struct KFusedDirect {
    float2* psi;
    uint64_t N;
    uint64_t n_tiles;
    int pos[10];               // tile bits ascending: 0..4 and the targets
    uint32_t toff[5];          // 1 << target j (T[0] = most significant row bit)
    const float* amat;
    uint32_t amat_stride;      // floats between batch rows' matrices (0: shared)
};

__device__ __forceinline__ uint32_t row_off(const KFusedDirect& a, int r)
{
    uint32_t o = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j)
        if ((r >> (4 - j)) & 1) o += a.toff[j];
    return o;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_fused_direct(KFusedDirect a)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5, c32 = lane & 31;
    float2* psi = a.psi + (uint64_t)blockIdx.y * a.N;
    const float* am = a.amat + (size_t)blockIdx.y * a.amat_stride;      // this row's matrix

    uint32_t ro_in[16], ro_out[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int r = MODE == 0 ? 2 * s + h : (s < 8 ? 8 * h + s : 16 + 8 * h + (s - 8));
        ro_in[s] = row_off(a, r) + c32;
        ro_out[s] = row_off(a, 8 * (s >> 2) + 4 * h + (s & 3)) + c32;
    }
    float afr[2][32];
    bf16x8 ahi[2][4], alo[2][4];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                // fragment-ordered copy after the two 64 x 64 parts:
                // element (b, q, lane, e) = A~[32 b + lane % 32][2 (4 q + e) + lane / 32]
                const float4 t4 = reinterpret_cast<const float4*>(am + 2 * 64 * 64)[(b * 8 + q) * 64 + lane];
                afr[b][4 * q] = t4.x;
                afr[b][4 * q + 1] = t4.y;
                afr[b][4 * q + 2] = t4.z;
                afr[b][4 * q + 3] = t4.w;
            }
    } else {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                // fragment-ordered BF16 copy after the two 64 x 64 parts: the 8
                // values of (b, s, part, lane) = part [32 b + lane % 32][16 s + 8 (lane / 32) + q]
                const u32x4* fb = reinterpret_cast<const u32x4*>(am + 2 * 64 * 64);
                ahi[b][s] = __builtin_bit_cast(bf16x8, fb[((b * 4 + s) * 2 + 0) * 64 + lane]);
                alo[b][s] = __builtin_bit_cast(bf16x8, fb[((b * 4 + s) * 2 + 1) * 64 + lane]);
            }
    }
    // tiles of this wave: w, w + W, w + 2W, ... (W waves in the grid); the
    // next tile's operands are loaded before this tile's products start, so
    // the load latency hides behind the matrix-core work
    const uint64_t waves_total = (uint64_t)gridDim.x * 4;
    uint64_t tile = xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
    float2 x[16];
    if (tile < a.n_tiles) {
        const float2* tp = psi + insert_zeros(tile, a.pos, 10);
#pragma unroll
        for (int s = 0; s < 16; ++s) x[s] = ld2(tp + ro_in[s]);
    }
    for (; tile < a.n_tiles; tile += waves_total) {
        float2* tp = psi + insert_zeros(tile, a.pos, 10);
        const uint64_t next = tile + waves_total;
        float2 xn[16];
        if (next < a.n_tiles) {
            const float2* np_ = psi + insert_zeros(next, a.pos, 10);
#pragma unroll
            for (int s = 0; s < 16; ++s) xn[s] = ld2(np_ + ro_in[s]);
        }
        f32x16 acc0 = {0}, acc1 = {0};
        if constexpr (MODE == 0) {
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[0][s], x[s].x, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[1][s], x[s].x, acc1, 0, 0, 0);
            }
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[0][16 + s], x[s].y, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[1][16 + s], x[s].y, acc1, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                float xh[8], xl[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) xh[q] = (s & 1) ? (s < 2 ? x[8 + q].x : x[8 + q].y)
                                                           : (s < 2 ? x[q].x : x[q].y);
                const bf16x8 bh = to_bf16(xh);
#pragma unroll
                for (int q = 0; q < 8; ++q) xl[q] = xh[q] - (float)bh[q];
                const bf16x8 bl = to_bf16(xl);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[0][s], bh, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[1][s], bh, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[0][s], bl, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[1][s], bl, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[0][s], bh, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[1][s], bh, acc1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) st2(tp + ro_out[q], make_float2(acc0[q], acc1[q]));
#pragma unroll
        for (int s = 0; s < 16; ++s) x[s] = xn[s];
    }
}

// Wide direct form for blocks whose five targets are all >= 6: a wave's tile
// is 32 rows x 64 columns (qubits 0..5), and every lane moves 16 bytes per
// access -- columns 2c and 2c+1 of one row. The two columns feed two
// independent products (column block A = even columns, B = odd columns), so
// the operand layout is unchanged and each memory instruction carries twice
// the bytes of the 8-byte form.
struct KFusedWide {
    float2* psi;
    uint64_t N;
    uint64_t n_tiles;
    int pos[11];               // tile bits ascending: 0..5 and the targets
    uint32_t toff[5];
    const float* amat;
    uint32_t amat_stride;      // floats between batch rows' matrices (0: shared)
};

template <int MODE>
__global__ __launch_bounds__(256) void k_fused_wide(KFusedWide a)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5, c32 = lane & 31;
    float2* psi = a.psi + (uint64_t)blockIdx.y * a.N;
    const float* am = a.amat + (size_t)blockIdx.y * a.amat_stride;      // this row's matrix

    auto roff = [&](int r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < 5; ++j)
            if ((r >> (4 - j)) & 1) o += a.toff[j];
        return o + 2 * c32;
    };
    uint32_t ro_in[16], ro_out[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        ro_in[s] = roff(MODE == 0 ? 2 * s + h : (s < 8 ? 8 * h + s : 16 + 8 * h + (s - 8)));
        ro_out[s] = roff(8 * (s >> 2) + 4 * h + (s & 3));
    }
    float afr[2][32];
    bf16x8 ahi[2][4], alo[2][4];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                // fragment-ordered copy after the two 64 x 64 parts:
                // element (b, q, lane, e) = A~[32 b + lane % 32][2 (4 q + e) + lane / 32]
                const float4 t4 = reinterpret_cast<const float4*>(am + 2 * 64 * 64)[(b * 8 + q) * 64 + lane];
                afr[b][4 * q] = t4.x;
                afr[b][4 * q + 1] = t4.y;
                afr[b][4 * q + 2] = t4.z;
                afr[b][4 * q + 3] = t4.w;
            }
    } else {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                // fragment-ordered BF16 copy after the two 64 x 64 parts: the 8
                // values of (b, s, part, lane) = part [32 b + lane % 32][16 s + 8 (lane / 32) + q]
                const u32x4* fb = reinterpret_cast<const u32x4*>(am + 2 * 64 * 64);
                ahi[b][s] = __builtin_bit_cast(bf16x8, fb[((b * 4 + s) * 2 + 0) * 64 + lane]);
                alo[b][s] = __builtin_bit_cast(bf16x8, fb[((b * 4 + s) * 2 + 1) * 64 + lane]);
            }
    }
    const uint64_t waves_total = (uint64_t)gridDim.x * 4;
    for (uint64_t tile = xcd_block(blockIdx.x, gridDim.x) * 4 + wave; tile < a.n_tiles; tile += waves_total) {
        float2* tp = psi + insert_zeros(tile, a.pos, 11);
        float4 x[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) x[s] = ld4(tp + ro_in[s]);
        f32x16 a0 = {0}, a1 = {0}, b0 = {0}, b1 = {0};
        if constexpr (MODE == 0) {
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[0][s], x[s].x, a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[1][s], x[s].x, a1, 0, 0, 0);
                b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[0][s], x[s].z, b0, 0, 0, 0);
                b1 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[1][s], x[s].z, b1, 0, 0, 0);
            }
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[0][16 + s], x[s].y, a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[1][16 + s], x[s].y, a1, 0, 0, 0);
                b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[0][16 + s], x[s].w, b0, 0, 0, 0);
                b1 = __builtin_amdgcn_mfma_f32_32x32x2f32(afr[1][16 + s], x[s].w, b1, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                // rows of k-step s: real parts of rows 8h+q (s=0), 16+8h+q (s=1),
                // imaginary parts of the same rows (s=2, 3)
                float xa[8], xb[8], la[8], lb[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float4 v = (s & 1) ? x[8 + q] : x[q];
                    xa[q] = s < 2 ? v.x : v.y;
                    xb[q] = s < 2 ? v.z : v.w;
                }
                const bf16x8 ah = to_bf16(xa), bh = to_bf16(xb);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    la[q] = xa[q] - (float)ah[q];
                    lb[q] = xb[q] - (float)bh[q];
                }
                const bf16x8 al = to_bf16(la), bl = to_bf16(lb);
                a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[0][s], ah, a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[1][s], ah, a1, 0, 0, 0);
                b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[0][s], bh, b0, 0, 0, 0);
                b1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[1][s], bh, b1, 0, 0, 0);
                a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[0][s], al, a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[1][s], al, a1, 0, 0, 0);
                b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[0][s], bl, b0, 0, 0, 0);
                b1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[1][s], bl, b1, 0, 0, 0);
                a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[0][s], ah, a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[1][s], ah, a1, 0, 0, 0);
                b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[0][s], bh, b0, 0, 0, 0);
                b1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[1][s], bh, b1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) st4(tp + ro_out[q], make_float4(a0[q], a1[q], b0[q], b1[q]));
    }
}

// Six-qubit blocks on the matrix cores (split BF16x3 only: at 2 x 6 = 12
// products per k-step the FP32 form would be bound by its MFMA rate). The
// complex 64 x 64 block is the real 128 x 128 embedding A~ = [[Mr, -Mi],
// [Mi, Mr]]; its BF16 hi and lo parts sit in LDS (rows padded to 136 so the
// 16-byte fragment reads of consecutive rows fall in different banks). A
// wave's tile is 64 rows (the targets, all >= 6) x 64 columns (qubits 0..5):
// each lane loads 16 B (two adjacent columns) of 32 rows -- rows 16 s' + 8 h
// + q, s' < 4, q < 8, the rows whose real and imaginary parts it supplies as
// the right operand of v_mfma_f32_32x32x16_bf16 -- and splits them into BF16
// hi/lo once. Output rows are produced in two halves (rows 0..31, then
// 32..63): real rows from A~ row block p, imaginary rows from block 2 + p,
// for the even and the odd columns (four accumulators); each half is stored
// as soon as it is complete, so only half of the accumulators are live.
// Row offsets split into a wave-uniform part and the lane's part as in the
// five-qubit wide form. Offsets fit 32 bits (n <= 32).
constexpr int kA6 = 136;               // padded row length of the 128 x 128 BF16 operand

struct KFusedWide6 {
    float2* psi;
    uint64_t N;
    uint64_t n_tiles;
    int pos[12];               // tile bits ascending: 0..5 and the six targets
    uint32_t toff[6];          // 1 << target j (T[0] = most significant row bit)
    const uint16_t* amat;      // BF16 bits: hi [128][kA6] then lo [128][kA6]
};

__global__ __launch_bounds__(256) void k_fused_wide6(KFusedWide6 a)
{
    __shared__ __align__(16) uint16_t as[2 * 128 * kA6];
    for (int i = threadIdx.x; i < 2 * 128 * kA6 / 8; i += 256)
        reinterpret_cast<uint4*>(as)[i] = reinterpret_cast<const uint4*>(a.amat)[i];
    __syncthreads();
    const __bf16* ahi = reinterpret_cast<const __bf16*>(as);
    const __bf16* alo = ahi + 128 * kA6;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = lane >> 5, c32 = lane & 31;
    float2* psi = a.psi + (uint64_t)blockIdx.y * a.N;
    // row r (6 bits, bit 5 = T[0]): uniform part of its offset
    auto urow = [&](int r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < 6; ++j)
            if ((r >> (5 - j)) & 1) o += a.toff[j];
        return o;
    };
    const uint32_t lane_in = 2 * c32 + (h ? a.toff[2] : 0u);    // bit 3 of the operand rows
    const uint32_t lane_out = 2 * c32 + (h ? a.toff[3] : 0u);   // bit 2 of the accumulator rows

    const uint64_t waves_total = (uint64_t)gridDim.x * 4;
    for (uint64_t tile = xcd_block(blockIdx.x, gridDim.x) * 4 + wave; tile < a.n_tiles; tile += waves_total) {
        // keep the block matrix in LDS: re-read its fragments every tile
        // instead of holding all 256 registers' worth across the loop
        asm volatile("" ::: "memory");
        float2* tp = psi + insert_zeros(tile, a.pos, 12);
        // right operands for k-step s (k = 16 s + 8 h + q): s < 4 real parts
        // of rows 16 s + 8 h + q, s >= 4 imaginary parts of rows 16 (s - 4) + 8 h + q;
        // [s][0] even column, [s][1] odd column
        bf16x8 bh[8][2], bl[8][2];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            float4 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = ld4(tp + urow(16 * g + q) + lane_in);
            float re0[8], re1[8], im0[8], im1[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                re0[q] = v[q].x;
                im0[q] = v[q].y;
                re1[q] = v[q].z;
                im1[q] = v[q].w;
            }
            auto split = [&](const float (&x)[8], bf16x8& hi, bf16x8& lo) {
                float l[8];
                hi = to_bf16(x);
#pragma unroll
                for (int q = 0; q < 8; ++q) l[q] = x[q] - (float)hi[q];
                lo = to_bf16(l);
            };
            split(re0, bh[g][0], bl[g][0]);
            split(re1, bh[g][1], bl[g][1]);
            split(im0, bh[4 + g][0], bl[4 + g][0]);
            split(im1, bh[4 + g][1], bl[4 + g][1]);
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            f32x16 re_e = {0}, im_e = {0}, re_o = {0}, im_o = {0};
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int k0 = 16 * s + 8 * h;
                const bf16x8 hr = *reinterpret_cast<const bf16x8*>(ahi + (32 * p + c32) * kA6 + k0);
                const bf16x8 lr = *reinterpret_cast<const bf16x8*>(alo + (32 * p + c32) * kA6 + k0);
                const bf16x8 hm = *reinterpret_cast<const bf16x8*>(ahi + (64 + 32 * p + c32) * kA6 + k0);
                const bf16x8 lm = *reinterpret_cast<const bf16x8*>(alo + (64 + 32 * p + c32) * kA6 + k0);
                re_e = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lr, bh[s][0], re_e, 0, 0, 0);
                im_e = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lm, bh[s][0], im_e, 0, 0, 0);
                re_o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lr, bh[s][1], re_o, 0, 0, 0);
                im_o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lm, bh[s][1], im_o, 0, 0, 0);
                re_e = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hr, bl[s][0], re_e, 0, 0, 0);
                im_e = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hm, bl[s][0], im_e, 0, 0, 0);
                re_o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hr, bl[s][1], re_o, 0, 0, 0);
                im_o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hm, bl[s][1], im_o, 0, 0, 0);
                re_e = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hr, bh[s][0], re_e, 0, 0, 0);
                im_e = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hm, bh[s][0], im_e, 0, 0, 0);
                re_o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hr, bh[s][1], re_o, 0, 0, 0);
                im_o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hm, bh[s][1], im_o, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q)
                st4(tp + urow(32 * p + 8 * (q >> 2) + (q & 3)) + lane_out, make_float4(re_e[q], im_e[q], re_o[q], im_o[q]));
        }
    }
}

// Plain FP32 vector form: one thread per column, the block matrix in LDS.
template <int K>
__global__ __launch_bounds__(256) void k_fused_valu(float2* psi, uint64_t N, uint64_t n_cols, int npos,
                                                    const int* __restrict__ pos_dev, const uint64_t* __restrict__ moff_dev,
                                                    const float2* __restrict__ m)
{
    constexpr int D = 1 << K;
    __shared__ float2 ms[D * D];
    __shared__ int pos[8];
    __shared__ uint64_t moff[D];
    for (int i = threadIdx.x; i < D * D; i += 256) ms[i] = m[i];
    if (threadIdx.x < npos) pos[threadIdx.x] = pos_dev[threadIdx.x];
    if (threadIdx.x < D) moff[threadIdx.x] = moff_dev[threadIdx.x];
    __syncthreads();
    float2* row = psi + (uint64_t)blockIdx.y * N;
    for (uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x; c < n_cols; c += (uint64_t)gridDim.x * 256) {
        const uint64_t base = insert_zeros(c, pos, npos);
        float2 x[D];
#pragma unroll
        for (int j = 0; j < D; ++j) x[j] = ld2(row + (base | moff[j]));
#pragma unroll 4
        for (int i = 0; i < D; ++i) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int j = 0; j < D; ++j) acc = cfma(ms[i * D + j], x[j], acc);
            st2(row + (base | moff[i]), acc);
        }
    }
}

// tiles per wave of the one-shot grids
constexpr uint64_t kOneShotTilesDirect = 4;
constexpr uint64_t kOneShotTilesLds = 8;

}  // namespace

void launch_fused_mfma(const FusedLaunch& f, hipStream_t st)
{
    const int nq = __builtin_ctzll(f.N);
    int lowest_target = 64;
    for (int j = 0; j < 5; ++j) lowest_target = std::min(lowest_target, f.targets[j]);
    if (lowest_target >= 6 && nq <= 32) {
        KFusedWide d{};
        d.psi = f.psi;
        d.N = f.N;
        d.n_tiles = 1ull << (nq - 11);
        int t5[5];
        for (int j = 0; j < 5; ++j) {
            t5[j] = f.targets[j];
            d.toff[j] = 1u << f.targets[j];
        }
        std::sort(t5, t5 + 5);
        for (int b = 0; b < 6; ++b) d.pos[b] = b;
        for (int b = 0; b < 5; ++b) d.pos[6 + b] = t5[b];
        d.amat = f.amat;
        d.amat_stride = f.amat_stride;
        // persistent grid of one workgroup per CU (276 registers per lane:
        // one wave per SIMD, so one workgroup per CU is resident); two per CU
        // (run one after the other) measured 1 % slower, one-shot grids of 2
        // to 16 tiles per wave 2-13 % slower
        const uint64_t want = (d.n_tiles + 3) / 4;
        const uint64_t cap = (uint64_t)device_info().cu_count;
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min(want, cap));
        if (f.mode == SV_FUSED_FP32_MFMA)
            hipLaunchKernelGGL(k_fused_wide<0>, dim3(grid, f.nrows), dim3(256), 0, st, d);
        else
            hipLaunchKernelGGL(k_fused_wide<1>, dim3(grid, f.nrows), dim3(256), 0, st, d);
        SV_HIP(hipGetLastError());
        return;
    }
    if (lowest_target >= 5 && nq <= 32) {
        KFusedDirect d{};
        d.psi = f.psi;
        d.N = f.N;
        d.n_tiles = 1ull << (nq - 10);
        int t5[5];
        for (int j = 0; j < 5; ++j) {
            t5[j] = f.targets[j];
            d.toff[j] = 1u << f.targets[j];
        }
        std::sort(t5, t5 + 5);
        for (int b = 0; b < 5; ++b) d.pos[b] = b;
        for (int b = 0; b < 5; ++b) d.pos[5 + b] = t5[b];
        d.amat = f.amat;
        d.amat_stride = f.amat_stride;
        // one-shot grid, four tiles per wave (the waves end as their tiles
        // are done; 3.05 / 2.99 ms per 30-qubit block in FP32 / BF16x3
        // against 3.48 / 3.24 with a persistent grid of two workgroups per
        // CU), never fewer workgroups than that persistent grid
        const uint64_t want = (d.n_tiles + 3) / 4;
        const uint64_t pers = std::min(want, (uint64_t)device_info().cu_count * 2);
        const uint64_t g = std::max(pers, want / kOneShotTilesDirect);
        const unsigned grid = (unsigned)std::max<uint64_t>(1, g);
        if (f.mode == SV_FUSED_FP32_MFMA)
            hipLaunchKernelGGL(k_fused_direct<0>, dim3(grid, f.nrows), dim3(256), 0, st, d);
        else
            hipLaunchKernelGGL(k_fused_direct<1>, dim3(grid, f.nrows), dim3(256), 0, st, d);
        SV_HIP(hipGetLastError());
        return;
    }
    KFused a{};
    a.psi = f.psi;
    a.N = f.N;
    const int n = __builtin_ctzll(f.N);
    a.n_tiles = 1ull << (n - 10);
    // tile bits: the 5 targets and the 5 lowest non-target qubits
    int cols[5], nc = 0;
    uint64_t tmask = 0;
    for (int j = 0; j < 5; ++j) tmask |= 1ull << f.targets[j];
    for (int q = 0; q < n && nc < 5; ++q)
        if (!((tmask >> q) & 1)) cols[nc++] = q;
    int np = 0;
    for (int q = 0; q < n; ++q)
        if (((tmask >> q) & 1) || (nc > 0 && q <= cols[4] && !((tmask >> q) & 1))) a.pos[np++] = q;
    // a.pos now lists every tile bit ascending (targets anywhere, columns = lowest non-targets)
    for (int b = 0; b < 10; ++b) {
        const int q = a.pos[b];
        a.bit_off64[b] = 1ull << q;
        a.bit_row[b] = 0;
        a.bit_col[b] = 0;
        for (int j = 0; j < 5; ++j)
            if (f.targets[j] == q) a.bit_row[b] = 1 << (4 - j);
        for (int c = 0; c < 5; ++c)
            if (cols[c] == q) a.bit_col[b] = 1 << c;
    }
    a.amat = f.amat;
    a.amat_stride = f.amat_stride;
    // one-shot grid, eight tiles per wave (3.24 / 3.16 ms per low-target
    // block of the 30-qubit brickwork plan in FP32 / BF16x3, against 3.29 /
    // 3.28 with the persistent grid of eight single-wave workgroups per CU),
    // never fewer workgroups than that persistent grid
    const uint64_t want = (a.n_tiles + kWaves - 1) / kWaves;
    const uint64_t pers = std::min(want, (uint64_t)device_info().cu_count * 8);
    const uint64_t g = std::max(pers, want / kOneShotTilesLds);
    const unsigned grid = (unsigned)std::max<uint64_t>(1, g);
    if (f.mode == SV_FUSED_FP32_MFMA)
        hipLaunchKernelGGL(k_fused<0>, dim3(grid, f.nrows), dim3(kWaves * 64), 0, st, a);
    else
        hipLaunchKernelGGL(k_fused<1>, dim3(grid, f.nrows), dim3(kWaves * 64), 0, st, a);
    SV_HIP(hipGetLastError());
}

size_t fused6_matrix_bytes() { return (size_t)2 * 128 * kA6 * sizeof(uint16_t); }

void fused6_layout(const float* embed, const float* embed_lo, uint16_t* out)
{
    // embed / embed_lo: row-major real 128 x 128 hi and lo parts (already
    // rounded to BF16 values); out: BF16 bits in the padded LDS layout
    auto bits = [](float x) {
        uint32_t u;
        std::memcpy(&u, &x, 4);
        return (uint16_t)(u >> 16);
    };
    for (int part = 0; part < 2; ++part) {
        const float* src = part == 0 ? embed : embed_lo;
        uint16_t* dst = out + (size_t)part * 128 * kA6;
        for (int r = 0; r < 128; ++r)
            for (int c = 0; c < kA6; ++c) dst[r * kA6 + c] = c < 128 ? bits(src[r * 128 + c]) : 0;
    }
}

void launch_fused_wide6(const Fused6Launch& f, hipStream_t st)
{
    const int nq = __builtin_ctzll(f.N);
    KFusedWide6 d{};
    d.psi = f.psi;
    d.N = f.N;
    d.n_tiles = 1ull << (nq - 12);
    int t6[6];
    for (int j = 0; j < 6; ++j) {
        t6[j] = f.targets[j];
        d.toff[j] = 1u << f.targets[j];
    }
    std::sort(t6, t6 + 6);
    for (int b = 0; b < 6; ++b) d.pos[b] = b;
    for (int b = 0; b < 6; ++b) d.pos[6 + b] = t6[b];
    d.amat = f.amat;
    // persistent grid: one workgroup (four waves) per CU; two would fit
    // (234 registers, 68 KiB of LDS each) but measured 7 % slower at 30 qubits
    const uint64_t want = (d.n_tiles + 3) / 4;
    const uint64_t cap = (uint64_t)device_info().cu_count;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min(want, cap));
    hipLaunchKernelGGL(k_fused_wide6, dim3(grid, f.nrows), dim3(256), 0, st, d);
    SV_HIP(hipGetLastError());
}

void launch_fused_valu(const FusedValuLaunch& f, hipStream_t st)
{
    const int n = __builtin_ctzll(f.N);
    const uint64_t n_cols = 1ull << (n - f.k);
    const uint64_t blocks = std::min<uint64_t>((n_cols + 255) / 256, (uint64_t)device_info().cu_count * 8);
    const dim3 gd((unsigned)std::max<uint64_t>(blocks, 1), f.nrows);
    switch (f.k) {
    case 1: hipLaunchKernelGGL(k_fused_valu<1>, gd, dim3(256), 0, st, f.psi, f.N, n_cols, f.k, f.pos, f.moff, f.m); break;
    case 2: hipLaunchKernelGGL(k_fused_valu<2>, gd, dim3(256), 0, st, f.psi, f.N, n_cols, f.k, f.pos, f.moff, f.m); break;
    case 3: hipLaunchKernelGGL(k_fused_valu<3>, gd, dim3(256), 0, st, f.psi, f.N, n_cols, f.k, f.pos, f.moff, f.m); break;
    case 4: hipLaunchKernelGGL(k_fused_valu<4>, gd, dim3(256), 0, st, f.psi, f.N, n_cols, f.k, f.pos, f.moff, f.m); break;
    default: hipLaunchKernelGGL(k_fused_valu<5>, gd, dim3(256), 0, st, f.psi, f.N, n_cols, f.k, f.pos, f.moff, f.m); break;
    }
    SV_HIP(hipGetLastError());
}

}  // namespace sv
