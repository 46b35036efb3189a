// k_adj_mfma.hip -- the blocked adjoint backward on the matrix cores.
//
// For a block of gates acting inside four qubits (local bit i = qubit q[i],
// ascending), the adjoint recursion of Sec. 4.4 regroups per block: with
// psi, lambda the vectors after the block and, for every column c (the 16
// amplitudes that differ only in the block's qubits), the block's
// correlation
//     S = sum_c psi_c lambda_c^*            (S[b][a] = sum_c psi_c[b] conj(lambda_c[a])),
// the derivative of gate k in the block is 2 Re Tr(X_k S) with
// X_k = W_k (dG_k G_k^*) W_k^* and W_k the block's gates after k (formed on
// the host in FP64); the vectors before the block are U_B^* psi and
// U_B^* lambda. One sweep per block therefore does two contractions:
//   * S as a real 32 x 32 product X_psi X_lambda^T over all columns (rows
//     0..15 the real parts, 16..31 the imaginary parts of a column), on
//     FP64 matrix cores (v_mfma_f64_16x16x4_f64): the FP32 data's products
//     are exact and the sums are FP64;
//   * the un-apply y = U_B^* x for both vectors, as the real 32 x 32 product
//     of [[Re M, -Im M], [Im M, Re M]] (M = U_B^*) with 32 columns at a time
//     on FP32 matrix cores (v_mfma_f32_32x32x2_f32).
// A wave takes 32 columns at a time; lane (h, u) (h = lane / 32) reads and
// writes amplitudes 8h .. 8h+7 of column u. For the correlation the columns
// are transposed through a per-wave LDS tile (the FP64 product wants a row
// per lane). Each wave keeps its S in registers; the workgroup sums its
// waves' S and writes one part, and a fixed tree of small kernels sums the
// parts (deterministic).
//
// The launch is one-shot: a wave takes a few groups (the next one's loads in
// flight while the current one is multiplied) and ends, and the grid covers
// the state once; loads and stores are non-temporal (every amplitude is
// touched once, in whole 128-byte lines). Measured on the bare access
// pattern (no arithmetic, 28 qubits, the next group's loads in flight): a
// persistent grid-stride loop took 1.62 ms non-temporal and 1.69 ms cached,
// one-shot with four groups per wave 1.55 ms (1.46 ms with each group's loads
// issued after the previous group's stores; in this kernel both orders
// measured the same).
#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kAmThreads = 256;
constexpr int kAmWaves = kAmThreads / 64;
// LDS tiles, one per vector and wave, 32 rows of real parts (0..15) and
// imaginary parts (16..31) of a group's 32 columns. Column form: rows of
// kTp = 34 floats (2 mod 32 banks), so the correlation's reads (16 rows x 2
// columns per half-wave) and the un-apply's (one row, 32 columns) fall on
// distinct banks. Memory-order form: rows of 32 floats with the column index
// XOR-swizzled by the row, entry (row, col) at row * 32 + (col ^ sw(row)),
// sw(row) = the four low row bits reversed into bits 4..1: the transposes'
// lanes vary the lowest bits of both the row (block bits) and the column (the
// lowest other qubits), and the reversal sends the row bits to the bank bits
// the column bits leave free, so those accesses, too, touch 32 distinct banks
// per half-wave (a padded pitch cannot serve every mix of row and column bits).
constexpr int kTp = 34;

template <bool COAL>
__device__ __forceinline__ int tix(int row, int col)
{
    if constexpr (COAL) {
        const int r = row & 15;
        const int sw = ((r & 1) << 4) | ((r & 2) << 2) | (r & 4) | ((r & 8) >> 2);
        return row * 32 + (col ^ sw);
    } else {
        return row * kTp + col;
    }
}

// A wave's own LDS writes complete before its following reads (and its
// reads before its following writes): wait for the LDS counter and keep the
// compiler from moving LDS accesses across.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);      // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wait for every vector memory operation of the wave (the operand fragments
// and the first group) before the loop: the loop's waits then count only the
// loop's own loads and stores, whatever order the prologue's loads took.
__device__ __forceinline__ void vm_drain()
{
    __builtin_amdgcn_s_waitcnt(0x0f70);      // vmcnt(0)
}

// The value unchanged, through an empty asm the compiler cannot see through.
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ float2* am_row(const Rows& r, int row)
{
    return row < r.nrow0 ? r.p0 + (uint64_t)row * r.N : r.p1 + (uint64_t)(row - r.nrow0) * r.N;
}

// COAL: a block qubit below 5. Consecutive columns are then up to 128 B
// apart, so the group's 512 amplitudes move in memory order instead: the
// group's nine varying address bits (the block's qubits and the five lowest
// other qubits) then include bits 0..5, so each load or store of the wave
// covers 512 contiguous bytes; the per-wave LDS tiles convert between
// memory order and the lane layout of the products. Three waves per SIMD
// (at most 168 registers; the compiler would take 172 in the column form).
template <bool COAL>
__global__ __launch_bounds__(kAmThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_adj_mfma(AdjMfmaLaunch a)
{
    // the psi and lambda tiles of every wave; at the end the same memory holds
    // the waves' S parts
    __shared__ float tiles[2][kAmWaves][32 * kTp];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);     // uniform: groups and bases are scalar
    const int h = lane >> 5, cu = lane & 31;
    const int row = blockIdx.y;
    float2* psi = am_row(a.psi, row);
    float2* lam = am_row(a.lam, row);
    float* tpw = tiles[0][w];
    float* tlw = tiles[1][w];
    float fr[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) fr[s] = a.frag[(size_t)row * a.frag_stride + lane * 16 + s];
    const int q0 = a.q[0], q1 = a.q[1], q2 = a.q[2], q3 = a.q[3];
    f64x4 s00 = {0, 0, 0, 0}, s10 = {0, 0, 0, 0}, s11 = {0, 0, 0, 0};
    const uint64_t groups = a.N >> 9;          // 32 columns of 16 amplitudes
    // column base of a group for column c (zeros at the block's qubits)
    auto column = [&](uint64_t grp, int c) {
        uint64_t u = grp * 32 + c;
        u = ((u >> q0) << (q0 + 1)) | (u & ((1ull << q0) - 1));
        u = ((u >> q1) << (q1 + 1)) | (u & ((1ull << q1) - 1));
        u = ((u >> q2) << (q2 + 1)) | (u & ((1ull << q2) - 1));
        return ((u >> q3) << (q3 + 1)) | (u & ((1ull << q3) - 1));
    };
    // Wave w of workgroup b takes groups (b gpw + i) kAmWaves + w, i < gpw:
    // a workgroup covers kAmWaves gpw consecutive groups. Each wave works
    // through its groups with its own LDS tiles, so only the wave itself has
    // to be in step between writing and reading them. The loop is rotated:
    // the next group's loads are issued before this group's stores, and the
    // tiles are refilled from them at the end of the iteration. Vector memory
    // operations count down in issue order, so waiting there for the loads
    // does not wait for the stores issued after them (refilling at the top of
    // the loop would: the stores of the previous group would sit between).
    uint64_t grp = (uint64_t)blockIdx.x * a.gpw * kAmWaves + w;
    constexpr uint64_t stride = kAmWaves;
    const uint64_t gend = grp + (uint64_t)a.gpw * stride < groups ? grp + (uint64_t)a.gpw * stride : groups;
    float2 x[8], l[8];
    // Three real products give S (Gauss): with the tile rows 0..15 the real
    // parts and 16..31 the imaginary parts,
    //   s00 += Re psi Re lam^T,  s11 += Im psi Im lam^T,
    //   s10 += (Re psi + Im psi)(Re lam - Im lam)^T,
    // so Re S = s00 + s11 and Im S = s10 - s00 + s11. The sums of two FP32
    // values are exact in FP64 (A lane holds row lane % 16 of step column
    // lane / 16).
    // The correlation's three FP64 chains and the un-apply of psi (below) run
    // interleaved step by step (four independent accumulator chains for the
    // matrix pipe); psi's results are written only after the loop, so the
    // correlation still reads the tile's values from before the block.
    auto correlate_unapply_psi = [&](int ln) {
        const int hh = ln >> 5, cc = ln & 31;
        f32x16 y = {0};
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            y = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[s], tpw[tix<COAL>(16 * (s & 1) + 8 * hh + (s >> 1), cc)], y, 0,
                                                     0, 0);
            if (s & 1) {
                const int st = s >> 1;
                const int kk = 4 * st + (ln >> 4), ii = ln & 15;
                const double a0 = tpw[tix<COAL>(ii, kk)], a1 = tpw[tix<COAL>(16 + ii, kk)];
                const double b0 = tlw[tix<COAL>(ii, kk)], b1 = tlw[tix<COAL>(16 + ii, kk)];
                s00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, s00, 0, 0, 0);
                s11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, s11, 0, 0, 0);
                s10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0 + a1, b0 - b1, s10, 0, 0, 0);
            }
        }
        return y;
    };
    // un-apply y = M x from a tile (step s: component s & 1 of amplitude
    // 8h + (s >> 1), tile row 16 (s & 1) + 8h + (s >> 1); output register r:
    // component r & 1 of amplitude 8h + (r >> 1))
    auto unapply = [&](const float* tw, int ln) {
        const int hh = ln >> 5, cc = ln & 31;
        f32x16 y = {0};
#pragma unroll
        for (int s = 0; s < 16; ++s)
            y = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[s], tw[tix<COAL>(16 * (s & 1) + 8 * hh + (s >> 1), cc)], y, 0,
                                                     0, 0);
        return y;
    };
    if constexpr (COAL) {
        // memory order: element m (9 bits) of a group sits at the group's base
        // plus m's bits deposited on the group's nine varying bits; lane and
        // pass k hold m = 64 k + lane. Depositing is linear over disjoint bits,
        // so the offset is the lane's part OR pass k's part (uniform), and the
        // tile entry (row j = the block bits, column c = the other varying
        // bits; tix(j, c) = 32 j + (c ^ sw(j)) with sw linear in j) is the
        // lane's entry XOR pass k's.
        const uint64_t qmask = (1ull << q0) | (1ull << q1) | (1ull << q2) | (1ull << q3);
        uint64_t cmask = 0;
        for (int b = 0, c = 0; c < 5; ++b)
            if (!((qmask >> b) & 1)) {
                cmask |= 1ull << b;
                ++c;
            }
        const uint64_t vmask = qmask | cmask;
        // position bits of the nine varying bits, ascending
        uint64_t vb[9];
        {
            uint64_t vm = vmask;
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                vb[r] = vm & (~vm + 1);
                vm ^= vb[r];
            }
        }
        auto entry = [&](uint64_t xo) {
            const int j = (int)((xo >> q0) & 1) | (int)(((xo >> q1) & 1) << 1) | (int)(((xo >> q2) & 1) << 2) |
                          (int)(((xo >> q3) & 1) << 3);
            int c = 0;
            uint64_t cm = cmask;
            for (int r = 0; r < 5; ++r) {
                const uint64_t low = cm & (~cm + 1);
                if (xo & low) c |= 1 << r;
                cm ^= low;
            }
            return tix<COAL>(j, c);
        };
        uint64_t mlane = 0;
#pragma unroll
        for (int r = 0; r < 6; ++r)
            if ((lane >> r) & 1) mlane |= vb[r];
        const int tl = entry(mlane);
        auto mk = [&](int k) { return ((k & 1) ? vb[6] : 0) | ((k & 2) ? vb[7] : 0) | ((k & 4) ? vb[8] : 0); };
        // the lane's byte offset: mlane < 512 (the six lowest varying bits are
        // below bit 9), so a 32-bit offset from a scalar base addresses it
        const uint32_t ml = (uint32_t)mlane * (uint32_t)sizeof(float2);
        auto at = [&](float2* p, uint64_t s) { return reinterpret_cast<float2*>(reinterpret_cast<char*>(p + s) + ml); };
        auto load = [&](uint64_t g) {
            const uint64_t base = column(g, 0);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                x[k] = ld2(at(psi, base | mk(k)));
                l[k] = ld2(at(lam, base | mk(k)));
            }
        };
        auto to_tiles = [&](int tli) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int ti = tli ^ entry(mk(k));
                tpw[ti] = x[k].x;
                tpw[ti + 16 * 32] = x[k].y;
                tlw[ti] = l[k].x;
                tlw[ti + 16 * 32] = l[k].y;
            }
        };
        if (grp < gend) {
            load(grp);
            to_tiles(tl);
        }
        vm_drain();
        for (; grp < gend; grp += stride) {
            // the swizzled tile entries are lane values XOR constants; taking
            // them from an opaque copy of the lane index each iteration keeps
            // the compiler from holding them all in registers across the loop
            const int ln = opaque(lane), tn = opaque(tl);
            const int hn = ln >> 5, cn = ln & 31;
            const uint64_t gn = grp + stride;
            if (gn < gend) load(gn);
            wave_lds_sync();
            // un-apply in place, one vector after the other: a lane's inputs
            // and outputs are the same tile entries (rows 8h + t and
            // 16 + 8h + t of column cu), and the wave's LDS accesses run in order
            f32x16 y = correlate_unapply_psi(ln);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                tpw[tix<COAL>(8 * hn + t, cn)] = y[2 * t];
                tpw[tix<COAL>(16 + 8 * hn + t, cn)] = y[2 * t + 1];
            }
            y = unapply(tlw, ln);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                tlw[tix<COAL>(8 * hn + t, cn)] = y[2 * t];
                tlw[tix<COAL>(16 + 8 * hn + t, cn)] = y[2 * t + 1];
            }
            wave_lds_sync();
            const uint64_t base = column(grp, 0);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int ti = tn ^ entry(mk(k));
                st2(at(psi, base | mk(k)), make_float2(tpw[ti], tpw[ti + 16 * 32]));
                st2(at(lam, base | mk(k)), make_float2(tlw[ti], tlw[ti + 16 * 32]));
            }
            wave_lds_sync();       // this group's tile reads are done before the next group's writes
            if (gn < gend) to_tiles(tn);
        }
    } else {
        // with every block qubit >= 5 the 32 columns of a group are 32
        // consecutive amplitudes: column(grp, cu) = column(grp, 0) | cu, so
        // amplitude 8h + t of a lane's column sits at a scalar base (the
        // group's, plus t's block bits) plus one per-lane offset
        const uint64_t lh = ((uint64_t)h << q3) | (uint64_t)cu;
        auto toff = [&](int t) {
            return ((uint64_t)(t & 1) << q0) | ((uint64_t)((t >> 1) & 1) << q1) | ((uint64_t)((t >> 2) & 1) << q2);
        };
        auto load = [&](uint64_t g) {
            const float2* pb = psi + column(g, 0);
            const float2* lb = lam + column(g, 0);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                x[t] = ld2(pb + toff(t) + lh);
                l[t] = ld2(lb + toff(t) + lh);
            }
        };
        // transpose: tile row = real index (amplitude 8h + t: row 8h + t real,
        // row 16 + 8h + t imaginary), tile column = column of the group
        auto to_tiles = [&]() {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                tpw[tix<COAL>(8 * h + t, cu)] = x[t].x;
                tpw[tix<COAL>(16 + 8 * h + t, cu)] = x[t].y;
                tlw[tix<COAL>(8 * h + t, cu)] = l[t].x;
                tlw[tix<COAL>(16 + 8 * h + t, cu)] = l[t].y;
            }
        };
        if (grp < gend) {
            load(grp);
            to_tiles();
        }
        vm_drain();
        for (; grp < gend; grp += stride) {
            const uint64_t gn = grp + stride;
            if (gn < gend) load(gn);
            wave_lds_sync();
            float2* pb = psi + column(grp, 0);
            float2* lb = lam + column(grp, 0);
            f32x16 y = correlate_unapply_psi(lane);
#pragma unroll
            for (int t = 0; t < 8; ++t) st2(pb + toff(t) + lh, make_float2(y[2 * t], y[2 * t + 1]));
            y = unapply(tlw, lane);
#pragma unroll
            for (int t = 0; t < 8; ++t) st2(lb + toff(t) + lh, make_float2(y[2 * t], y[2 * t + 1]));
            wave_lds_sync();        // this group's tile reads are done before the next group's writes
            if (gn < gend) to_tiles();
        }
    }
    // the workgroup's part: Re S (16 x 16, row-major) then Im S, the waves'
    // values summed in wave order through LDS (the tiles are free now); the
    // FP64 product's output register r of lane l is row 4r + l / 16, column
    // l % 16 of a 16 x 16 product
    __syncthreads();       // every wave is done with its tiles
    double* red = reinterpret_cast<double*>(&tiles[0][0][0]);    // [kAmWaves][kAmPart]
    static_assert(sizeof(tiles) >= kAmWaves * kAmPart * sizeof(double), "the waves' parts fit the tiles");
    const int col = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ri = 4 * r + (lane >> 4);
        double* rw = red + w * kAmPart;
        rw[ri * 16 + col] = s00[r] + s11[r];
        rw[256 + ri * 16 + col] = s10[r] - s00[r] + s11[r];
    }
    __syncthreads();
    double* sp = a.spart + ((size_t)row * gridDim.x + blockIdx.x) * kAmPart;
    for (int e = threadIdx.x; e < kAmPart; e += kAmThreads) {
        double acc = red[e];
#pragma unroll
        for (int v = 1; v < kAmWaves; ++v) acc += red[v * kAmPart + e];
        sp[e] = acc;
    }
}

// Fixed-order sum of the workgroups' parts: level by level, part c of the
// next level is the sum of parts 64 c .. 64 c + 63 of this one (each thread
// one of the kAmPart entries, eight accumulators in a fixed pattern keep
// eight loads in flight), until one is left; the last level writes S_real in
// its four-quadrant form [Re psi Re lam^T, Re psi Im lam^T; Im psi Re lam^T,
// Im psi Im lam^T] with Re S in the upper-left block, Im S in the lower-left
// one and zeros elsewhere, so that Re S = upper-left + lower-right and
// Im S = lower-left - upper-right.
constexpr int kAmRun = 64;

__device__ __forceinline__ double sum_run(const double* __restrict__ p, int count)
{
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int v = 0;
    for (; v + 8 <= count; v += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += p[(size_t)(v + u) * kAmPart];
    for (; v < count; ++v) acc[0] += p[(size_t)v * kAmPart];
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

__global__ __launch_bounds__(kAmThreads) void k_adj_mfma_sum(const double* __restrict__ in, int parts,
                                                             double* __restrict__ out)
{
    const int c = blockIdx.x >> 1, row = blockIdx.y;
    const int e = (blockIdx.x & 1) * kAmThreads + threadIdx.x;
    const int nout = (parts + kAmRun - 1) / kAmRun;
    const int p0 = c * kAmRun, cnt = min(kAmRun, parts - p0);
    out[((size_t)row * nout + c) * kAmPart + e] = sum_run(in + ((size_t)row * parts + p0) * kAmPart + e, cnt);
}

__global__ __launch_bounds__(kAmThreads) void k_adj_mfma_final(const double* __restrict__ in, int parts,
                                                               double* __restrict__ s_out)
{
    const int row = blockIdx.y;
    const int e = blockIdx.x * kAmThreads + threadIdx.x;      // 0..511: Re S entries, then Im S
    const double v = sum_run(in + (size_t)row * parts * kAmPart + e, parts);
    const int i = (e & 255) >> 4, j = e & 15;
    double* o = s_out + (size_t)row * 1024;
    if (e < 256) {
        o[i * 32 + j] = v;               // upper-left: Re S
        o[i * 32 + 16 + j] = 0.0;        // upper-right
    } else {
        o[(16 + i) * 32 + j] = v;        // lower-left: Im S
        o[(16 + i) * 32 + 16 + j] = 0.0; // lower-right
    }
}

}  // namespace

// Groups per wave and workgroups per row: kAmMinGpw groups per wave (the
// parts cost 4 KiB per workgroup), fewer while the launch would not fill the
// chip once (three resident workgroups per CU), more while the parts of all
// rows would pass kAmMaxParts.
AdjMfmaShape adj_mfma_shape(int n, int rows, int min_gpw)
{
    const uint64_t groups = std::max<uint64_t>(1, (1ull << n) >> 9);
    const uint64_t r = (uint64_t)std::max(rows, 1);
    const uint64_t fill = (uint64_t)device_info().cu_count * 3;
    auto wgs = [&](uint64_t g) { return (groups + kAmWaves * g - 1) / (kAmWaves * g); };
    uint64_t gpw = (uint64_t)std::max(1, min_gpw);
    while (gpw > 1 && wgs(gpw) * r < fill) gpw /= 2;
    while (wgs(gpw) * r > kAmMaxParts) gpw *= 2;
    return AdjMfmaShape{(int)wgs(gpw), (int)gpw};
}

// doubles of the parts and of the two level buffers for `rows` rows at
// `grid` workgroups per row
uint64_t adj_mfma_part_doubles(int grid, int rows)
{
    const uint64_t lvl = ((uint64_t)grid + kAmRun - 1) / kAmRun;
    return (uint64_t)rows * ((uint64_t)grid + 2 * lvl) * kAmPart;
}

void launch_adj_mfma(const AdjMfmaLaunch& a, int rows, double* s_out, hipStream_t st)
{
    if (a.q[0] < 5) hipLaunchKernelGGL(k_adj_mfma<true>, dim3(a.grid, rows), dim3(kAmThreads), 0, st, a);
    else hipLaunchKernelGGL(k_adj_mfma<false>, dim3(a.grid, rows), dim3(kAmThreads), 0, st, a);
    SV_HIP(hipGetLastError());
    static_assert(2 * kAmThreads == kAmPart, "the sums give each thread one of the part's entries");
    const uint64_t lvl = ((uint64_t)a.grid + kAmRun - 1) / kAmRun;
    double* buf[2] = {a.spart + (uint64_t)rows * a.grid * kAmPart, a.spart + (uint64_t)rows * (a.grid + lvl) * kAmPart};
    const double* in = a.spart;
    int parts = a.grid, b = 0;
    while (parts > kAmRun) {
        const int nout = (parts + kAmRun - 1) / kAmRun;
        hipLaunchKernelGGL(k_adj_mfma_sum, dim3(2 * nout, rows), dim3(kAmThreads), 0, st, in, parts, buf[b]);
        SV_HIP(hipGetLastError());
        in = buf[b];
        b ^= 1;
        parts = nout;
    }
    hipLaunchKernelGGL(k_adj_mfma_final, dim3(2, rows), dim3(kAmThreads), 0, st, in, parts, s_out);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
