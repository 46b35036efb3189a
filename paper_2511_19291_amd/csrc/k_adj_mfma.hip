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
// per lane). Each wave keeps its S in registers and writes it once; a
// second kernel sums the waves' S in a fixed order (deterministic).
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

__device__ __forceinline__ float2* am_row(const Rows& r, int row)
{
    return row < r.nrow0 ? r.p0 + (uint64_t)row * r.N : r.p1 + (uint64_t)(row - r.nrow0) * r.N;
}

// COAL: a block qubit below 5. Consecutive columns are then up to 128 B
// apart, so the group's 512 amplitudes move in memory order instead: the
// group's nine varying address bits (the block's qubits and the five lowest
// other qubits) then include bits 0..5, so each load or store of the wave
// covers 512 contiguous bytes; the per-wave LDS tiles convert between
// memory order and the lane layout of the products.
template <bool COAL>
__global__ __launch_bounds__(kAmThreads) void k_adj_mfma(AdjMfmaLaunch a)
{
    // the psi and lambda tiles of every wave; at the end the same memory holds
    // the waves' S parts (4 x 1024 doubles = 32 KiB <= 2 x 4 x 32 x 33 floats)
    __shared__ float tiles[2][kAmWaves][32 * kTp];
    static_assert(sizeof(tiles) >= kAmWaves * 1024 * sizeof(double), "S parts fit the tiles");
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
    const uint64_t stride = (uint64_t)gridDim.x * kAmWaves;
    // column base of a group for column c (zeros at the block's qubits)
    auto column = [&](uint64_t grp, int c) {
        uint64_t u = grp * 32 + c;
        u = ((u >> q0) << (q0 + 1)) | (u & ((1ull << q0) - 1));
        u = ((u >> q1) << (q1 + 1)) | (u & ((1ull << q1) - 1));
        u = ((u >> q2) << (q2 + 1)) | (u & ((1ull << q2) - 1));
        return ((u >> q3) << (q3 + 1)) | (u & ((1ull << q3) - 1));
    };
    // Three real products give S (Gauss): with the tile rows 0..15 the real
    // parts and 16..31 the imaginary parts,
    //   s00 += Re psi Re lam^T,  s11 += Im psi Im lam^T,
    //   s10 += (Re psi + Im psi)(Re lam - Im lam)^T,
    // so Re S = s00 + s11 and Im S = s10 - s00 + s11. The sums of two FP32
    // values are exact in FP64 (A lane holds row lane % 16 of step column
    // lane / 16).
    auto correlate = [&]() {
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int kk = 4 * st + (lane >> 4), ii = lane & 15;
            const double a0 = tpw[tix<COAL>(ii, kk)], a1 = tpw[tix<COAL>(16 + ii, kk)];
            const double b0 = tlw[tix<COAL>(ii, kk)], b1 = tlw[tix<COAL>(16 + ii, kk)];
            s00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, s00, 0, 0, 0);
            s11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, s11, 0, 0, 0);
            s10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0 + a1, b0 - b1, s10, 0, 0, 0);
        }
    };
    uint64_t grp = (uint64_t)blockIdx.x * kAmWaves + w;
    if constexpr (COAL) {
        // memory order: element m (9 bits) of a group sits at the group's base
        // plus m's bits deposited on the group's nine varying bits; lane and
        // pass k hold m = 64 k + lane. mo: its offset; ti: its tile entry.
        const uint64_t qmask = (1ull << q0) | (1ull << q1) | (1ull << q2) | (1ull << q3);
        uint64_t cmask = 0;
        for (int b = 0, c = 0; c < 5; ++b)
            if (!((qmask >> b) & 1)) {
                cmask |= 1ull << b;
                ++c;
            }
        const uint64_t vmask = qmask | cmask;
        uint64_t mo[8];
        int ti[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            uint32_t m = 64 * k + lane;
            uint64_t x = 0, vm = vmask;
            for (int r = 0; r < 9; ++r) {
                const uint64_t low = vm & (~vm + 1);
                if ((m >> r) & 1) x |= low;
                vm ^= low;
            }
            int j = 0, c = 0;
            j |= (int)((x >> q0) & 1) | (int)(((x >> q1) & 1) << 1) | (int)(((x >> q2) & 1) << 2) |
                 (int)(((x >> q3) & 1) << 3);
            uint64_t cm = cmask;
            for (int r = 0; r < 5; ++r) {
                const uint64_t low = cm & (~cm + 1);
                if (x & low) c |= 1 << r;
                cm ^= low;
            }
            mo[k] = x;
            ti[k] = tix<COAL>(j, c);
        }
        for (; grp < groups; grp += stride) {
            const uint64_t base = column(grp, 0);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float2 v = psi[base | mo[k]], e = lam[base | mo[k]];
                tpw[ti[k]] = v.x;
                tpw[ti[k] + 16 * 32] = v.y;
                tlw[ti[k]] = e.x;
                tlw[ti[k] + 16 * 32] = e.y;
            }
            wave_lds_sync();
            correlate();
            // un-apply in place, one vector after the other: a lane's inputs
            // and outputs are the same tile entries (rows 8h + t and
            // 16 + 8h + t of column cu), and the wave's LDS accesses run in order
            f32x16 y = {0};
#pragma unroll
            for (int s = 0; s < 16; ++s)
                y = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[s], tpw[tix<COAL>(16 * (s & 1) + 8 * h + (s >> 1), cu)], y, 0, 0,
                                                         0);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                tpw[tix<COAL>(8 * h + t, cu)] = y[2 * t];
                tpw[tix<COAL>(16 + 8 * h + t, cu)] = y[2 * t + 1];
            }
            y = f32x16{0};
#pragma unroll
            for (int s = 0; s < 16; ++s)
                y = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[s], tlw[tix<COAL>(16 * (s & 1) + 8 * h + (s >> 1), cu)], y, 0, 0,
                                                         0);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                tlw[tix<COAL>(8 * h + t, cu)] = y[2 * t];
                tlw[tix<COAL>(16 + 8 * h + t, cu)] = y[2 * t + 1];
            }
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                psi[base | mo[k]] = make_float2(tpw[ti[k]], tpw[ti[k] + 16 * 32]);
                lam[base | mo[k]] = make_float2(tlw[ti[k]], tlw[ti[k] + 16 * 32]);
            }
            wave_lds_sync();
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
        // the next group's columns are loaded (into the same registers) while
        // this group's products run: the products read their inputs from the
        // LDS tiles. Each wave works through its own groups (its LDS tiles are
        // its own, so only the wave itself has to be in step between writing
        // and reading them).
        float2 x[8], l[8];
        if (grp < groups) {
            const float2* pb = psi + column(grp, 0);
            const float2* lb = lam + column(grp, 0);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                x[t] = pb[toff(t) + lh];
                l[t] = lb[toff(t) + lh];
            }
        }
        for (; grp < groups; grp += stride) {
            // transpose: tile row = real index (amplitude 8h + t: row 8h + t
            // real, row 16 + 8h + t imaginary), tile column = column of the group
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                tpw[tix<COAL>(8 * h + t, cu)] = x[t].x;
                tpw[tix<COAL>(16 + 8 * h + t, cu)] = x[t].y;
                tlw[tix<COAL>(8 * h + t, cu)] = l[t].x;
                tlw[tix<COAL>(16 + 8 * h + t, cu)] = l[t].y;
            }
            const uint64_t gn = grp + stride;
            if (gn < groups) {
                const float2* pn = psi + column(gn, 0);
                const float2* ln = lam + column(gn, 0);
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    x[t] = pn[toff(t) + lh];
                    l[t] = ln[toff(t) + lh];
                }
            }
            wave_lds_sync();
            correlate();
            // un-apply y = M x, one vector after the other (step s: component
            // s & 1 of amplitude 8h + (s >> 1), tile row 16 (s & 1) + 8h + (s >> 1);
            // output register r: component r & 1 of amplitude 8h + (r >> 1))
            float2* pb = psi + column(grp, 0);
            float2* lb = lam + column(grp, 0);
            f32x16 y = {0};
#pragma unroll
            for (int s = 0; s < 16; ++s)
                y = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[s], tpw[tix<COAL>(16 * (s & 1) + 8 * h + (s >> 1), cu)], y, 0, 0,
                                                         0);
#pragma unroll
            for (int t = 0; t < 8; ++t) pb[toff(t) + lh] = make_float2(y[2 * t], y[2 * t + 1]);
            y = f32x16{0};
#pragma unroll
            for (int s = 0; s < 16; ++s)
                y = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[s], tlw[tix<COAL>(16 * (s & 1) + 8 * h + (s >> 1), cu)], y, 0, 0,
                                                         0);
#pragma unroll
            for (int t = 0; t < 8; ++t) lb[toff(t) + lh] = make_float2(y[2 * t], y[2 * t + 1]);
            wave_lds_sync();        // this group's tile reads are done before the next group's writes
        }
    }
    // the workgroup's S_real (32 x 32, row-major): the waves' parts summed in
    // wave order through LDS (the tiles are free now); the FP64 product's
    // output register r of lane l is row 4r + l / 16, column l % 16 of a
    // 16 x 16 part
    __syncthreads();       // every wave is done with its tiles
    double* red = reinterpret_cast<double*>(&tiles[0][0][0]);    // [kAmWaves][1024]
    const int col = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ri = 4 * r + (lane >> 4);
        double* rw = red + w * 1024;
        // S_real in its four-quadrant form: [Re psi Re lam^T, Re psi Im lam^T;
        // Im psi Re lam^T, Im psi Im lam^T], here with the lower-left block
        // holding Im S + upper-right (so that Im S = lower-left - upper-right)
        rw[ri * 32 + col] = s00[r];
        rw[ri * 32 + 16 + col] = 0.0;
        rw[(16 + ri) * 32 + col] = s10[r] - s00[r] + s11[r];
        rw[(16 + ri) * 32 + 16 + col] = s11[r];
    }
    __syncthreads();
    double* sp = a.spart + ((size_t)row * gridDim.x + blockIdx.x) * 1024;
    for (int e = threadIdx.x; e < 1024; e += kAmThreads) {
        double acc = red[e];
#pragma unroll
        for (int v = 1; v < kAmWaves; ++v) acc += red[v * 1024 + e];
        sp[e] = acc;
    }
}

// Two-level fixed-order sum of the workgroups' S_real. Level 1: chunk c of
// the workgroups (in order) per row, one element per thread, so that a launch
// has kAmChunks x 4 workgroups per row; level 2: the chunks in order. Four
// accumulators in a fixed pattern keep four loads in flight per thread.
constexpr int kAmChunks = 64;

__device__ __forceinline__ double sum_strided(const double* __restrict__ p, int count, size_t stride)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int v = 0;
    for (; v + 4 <= count; v += 4) {
        a0 += p[(size_t)v * stride];
        a1 += p[(size_t)(v + 1) * stride];
        a2 += p[(size_t)(v + 2) * stride];
        a3 += p[(size_t)(v + 3) * stride];
    }
    for (; v < count; ++v) a0 += p[(size_t)v * stride];
    return (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(kAmThreads) void k_adj_mfma_reduce1(const double* __restrict__ spart, int parts,
                                                                 double* __restrict__ mid)
{
    const int c = blockIdx.x >> 2, row = blockIdx.y;
    const int e = (blockIdx.x & 3) * kAmThreads + threadIdx.x;
    const int per = (parts + kAmChunks - 1) / kAmChunks;
    const int p0 = min(parts, c * per), p1 = min(parts, p0 + per);
    const double* p = spart + ((size_t)row * parts + p0) * 1024 + e;
    mid[((size_t)row * kAmChunks + c) * 1024 + e] = sum_strided(p, p1 - p0, 1024);
}

__global__ __launch_bounds__(kAmThreads) void k_adj_mfma_reduce2(const double* __restrict__ mid,
                                                                 double* __restrict__ out)
{
    const int row = blockIdx.y;
    const int e = blockIdx.x * kAmThreads + threadIdx.x;
    out[(size_t)row * 1024 + e] = sum_strided(mid + (size_t)row * kAmChunks * 1024 + e, kAmChunks, 1024);
}

}  // namespace

int adj_mfma_grid(int n)
{
    static int resident = 0;
    if (resident == 0) {
        int nb = 0;
        SV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_adj_mfma<false>),
                                                             kAmThreads, 0));
        resident = std::max(nb, 1);
    }
    const uint64_t groups = (1ull << n) >> 9;
    const uint64_t wgs = (groups + kAmWaves - 1) / kAmWaves;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(wgs, (uint64_t)device_info().cu_count * resident));
}

// doubles of the S parts for `rows` rows at `grid` workgroups per row
uint64_t adj_mfma_part_doubles(int grid, int rows)
{
    return (uint64_t)rows * ((uint64_t)grid + kAmChunks) * 1024;
}

void launch_adj_mfma(const AdjMfmaLaunch& a, int rows, double* s_out, hipStream_t st)
{
    if (a.q[0] < 5) hipLaunchKernelGGL(k_adj_mfma<true>, dim3(a.grid, rows), dim3(kAmThreads), 0, st, a);
    else hipLaunchKernelGGL(k_adj_mfma<false>, dim3(a.grid, rows), dim3(kAmThreads), 0, st, a);
    SV_HIP(hipGetLastError());
    double* mid = a.spart + (uint64_t)rows * a.grid * 1024;
    static_assert(4 * kAmThreads == 1024, "the reductions give each thread one of the 1024 entries");
    hipLaunchKernelGGL(k_adj_mfma_reduce1, dim3(kAmChunks * 4, rows), dim3(kAmThreads), 0, st, a.spart, a.grid,
                       mid);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_adj_mfma_reduce2, dim3(4, rows), dim3(kAmThreads), 0, st, mid, s_out);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
