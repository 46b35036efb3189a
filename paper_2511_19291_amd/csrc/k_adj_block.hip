// k_adj_block.hip -- the adjoint backward over a block of gates in one sweep.
//
// The per-gate backward (k_adjoint.hip) un-applies one gate per sweep over
// psi and lambda (Sec. 4.4: the layer input is recomputed as x = U^* y). When
// a run of gates acts on at most LB = 3, 4 or 5 qubits, all of its steps are
// local to the 2^LB amplitudes that differ only in those qubits (a column):
// one sweep loads each column of psi_l and lambda_l into registers, and for
// the block's gates from last to first adds the derivative terms and
// un-applies U^* from both vectors, then stores the column back. The
// gradient terms and the recovered states are those of the per-gate
// recursion, gate by gate; the bytes moved per block are those of one
// per-gate step.
//
// Per gate (uniform over the launch): U^* is applied as a dense matrix, as a
// diagonal, or as a plain exchange of the two members (X); a derivative is
// either general, 2 Re <lam| G |psi> with G = dU/dtheta U^* in FP64, or, for
// a Pauli rotation exp(-i theta P / 2) (P = X, Y, Z, XX, YY, ZZ, possibly
// controlled), G = -i P / 2, i.e. Re <lam|G|psi> = Im <lam|P|psi> / 2, whose
// pairwise products are formed in FP32 (the rounding of the complex64 data
// itself) and accumulated in FP64.
//
// Columns: local bit i is qubit q[i] (ascending); column c takes the other
// qubits' bits from c. A wave handles 64 consecutive columns at a time, so
// when qubit 0 is not in the block a load instruction reads 512 contiguous
// bytes. Each derivative's column terms are summed across the wave with a
// fixed shuffle tree and added by lane 0 to the wave's slot in LDS (one
// writer per slot, in gate and column order): the sums are deterministic.
#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

namespace {

__device__ __forceinline__ float2* arow(const Rows& r, int row)
{
    return row < r.nrow0 ? r.p0 + (uint64_t)row * r.N : r.p1 + (uint64_t)(row - r.nrow0) * r.N;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Im(conj(a) b) and Re(conj(a) b) in FP32
__device__ __forceinline__ float im_cb(float2 a, float2 b) { return fmaf(a.x, b.y, -a.y * b.x); }
__device__ __forceinline__ float re_cb(float2 a, float2 b) { return fmaf(a.x, b.x, a.y * b.y); }

// Re sum_i conj(l_i) (G x)_i over a group of D amplitudes (FP64)
template <int D>
__device__ __forceinline__ double grad_general(const double2* __restrict__ g, const float2 (&x)[D], const float2 (&l)[D])
{
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double mr = 0.0, mi = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double2 gij = g[i * D + j];
            mr += gij.x * x[j].x - gij.y * x[j].y;
            mi += gij.x * x[j].y + gij.y * x[j].x;
        }
        acc += (double)l[i].x * mr + (double)l[i].y * mi;
    }
    return acc;
}

// Im <l|P|x> over a group for the Pauli P (compile-time): 1 X, 2 Y, 3 Z
// (one target) or 4 XX, 5 YY, 6 ZZ (two targets; member r = (bit of t0,
// bit of t1): XX maps r to 3 - r, YY the same with signs -, +, +, -, ZZ is
// diagonal with signs (-1)^popcount(r))
template <int PK, int D>
__device__ __forceinline__ float grad_pauli(const float2 (&x)[D], const float2 (&l)[D])
{
    if constexpr (PK == 1) return im_cb(l[0], x[1]) + im_cb(l[1], x[0]);
    else if constexpr (PK == 2) return -re_cb(l[0], x[1]) + re_cb(l[1], x[0]);
    else if constexpr (PK == 3) return im_cb(l[0], x[0]) - im_cb(l[1], x[1]);
    else if constexpr (PK == 4) return im_cb(l[0], x[3]) + im_cb(l[1], x[2]) + im_cb(l[2], x[1]) + im_cb(l[3], x[0]);
    else if constexpr (PK == 5) return -im_cb(l[0], x[3]) + im_cb(l[1], x[2]) + im_cb(l[2], x[1]) - im_cb(l[3], x[0]);
    else return im_cb(l[0], x[0]) - im_cb(l[1], x[1]) - im_cb(l[2], x[2]) + im_cb(l[3], x[3]);
}

template <int D>
__device__ __forceinline__ void unapply_dense(const float2 (&u)[D * D], float2 (&x)[D])
{
    float2 y[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float2 acc = cmul(u[i * D], x[0]);
#pragma unroll
        for (int j = 1; j < D; ++j) acc = cfma(u[i * D + j], x[j], acc);
        y[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = y[i];
}

// Gate modes (uniform over a launch, resolved before the column loop so the
// unrolled group loop carries no branches): exchange (X, controlled or not,
// no parameter), dense U^* without derivative, dense U^* with the Pauli
// derivative PK, dense U^* with general FP64 derivatives.
enum { kModeExchange = 0, kModeDense = 1, kModePauli = 2, kModeGeneral = 3 };

// One gate on the column: derivative terms (on psi_l, lambda_l), then
// psi <- U^* psi, lambda <- U^* lambda. Groups: the amplitudes whose local
// index differs only in the target bits, with every control bit set.
template <int L, int NT, int T0, int T1, int MODE, int PK>
__device__ __forceinline__ void column_gate(const AdjBlockGate& G, float2 (&x)[L], float2 (&l)[L], double (&part)[3])
{
    constexpr int D = 1 << NT;
    constexpr int tm = NT == 1 ? (1 << T0) : ((1 << T0) | (1 << T1));
    const int cm = G.cmask;
    float2 u[D * D];
    if constexpr (MODE != kModeExchange) {
#pragma unroll
        for (int q = 0; q < D * D; ++q) u[q] = G.u[q];
    }
    float pp = 0.f;
    double gacc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < L; ++j) {
        if (j & tm) continue;
        if ((j & cm) != cm) continue;
        int idx[D];
        if constexpr (NT == 1) {
            idx[0] = j;
            idx[1] = j | (1 << T0);
        } else {
            idx[0] = j;
            idx[1] = j | (1 << T1);
            idx[2] = j | (1 << T0);
            idx[3] = j | (1 << T0) | (1 << T1);
        }
        float2 xs[D], ls[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            xs[r] = x[idx[r]];
            ls[r] = l[idx[r]];
        }
        if constexpr (MODE == kModePauli) pp += grad_pauli<PK, D>(xs, ls);
        if constexpr (MODE == kModeGeneral) {
#pragma unroll
            for (int d = 0; d < (NT == 1 ? 3 : 1); ++d)
                if (d < G.nd) gacc[d] += grad_general<D>(G.g[d], xs, ls);
        }
        if constexpr (MODE == kModeExchange) {
            x[idx[0]] = xs[1];
            x[idx[1]] = xs[0];
            l[idx[0]] = ls[1];
            l[idx[1]] = ls[0];
        } else {
            unapply_dense<D>(u, xs);
            unapply_dense<D>(u, ls);
#pragma unroll
            for (int r = 0; r < D; ++r) {
                x[idx[r]] = xs[r];
                l[idx[r]] = ls[r];
            }
        }
    }
    if constexpr (MODE == kModePauli) part[0] = 0.5 * (double)pp;
    if constexpr (MODE == kModeGeneral)
#pragma unroll
        for (int d = 0; d < 3; ++d) part[d] = gacc[d];
}

template <int L, int NT, int T0, int T1>
__device__ __forceinline__ void gate_modes(const AdjBlockGate& G, float2 (&x)[L], float2 (&l)[L], double (&part)[3])
{
    if constexpr (NT == 1) {
        if (G.nd == 0) {
            if (G.form == 2) column_gate<L, 1, T0, 0, kModeExchange, 0>(G, x, l, part);
            else column_gate<L, 1, T0, 0, kModeDense, 0>(G, x, l, part);
        } else {
            switch (G.pauli) {
            case 1: column_gate<L, 1, T0, 0, kModePauli, 1>(G, x, l, part); break;
            case 2: column_gate<L, 1, T0, 0, kModePauli, 2>(G, x, l, part); break;
            case 3: column_gate<L, 1, T0, 0, kModePauli, 3>(G, x, l, part); break;
            default: column_gate<L, 1, T0, 0, kModeGeneral, 0>(G, x, l, part); break;
            }
        }
    } else {
        if (G.nd == 0) {
            column_gate<L, 2, T0, T1, kModeDense, 0>(G, x, l, part);
        } else {
            // the two-target kinds with a parameter are the Pauli rotations
            // RXX, RYY, RZZ (the host refuses anything else)
            switch (G.pauli) {
            case 4: column_gate<L, 2, T0, T1, kModePauli, 4>(G, x, l, part); break;
            case 5: column_gate<L, 2, T0, T1, kModePauli, 5>(G, x, l, part); break;
            default: column_gate<L, 2, T0, T1, kModePauli, 6>(G, x, l, part); break;
            }
        }
    }
}

template <int L>
__device__ __forceinline__ void dispatch_gate(const AdjBlockGate& G, float2 (&x)[L], float2 (&l)[L], double (&part)[3])
{
    if (G.nt == 1) {
        switch (G.t0) {
        case 0: gate_modes<L, 1, 0, 0>(G, x, l, part); break;
        case 1: gate_modes<L, 1, 1, 0>(G, x, l, part); break;
        case 2: gate_modes<L, 1, 2, 0>(G, x, l, part); break;
        case 3:
            if constexpr (L >= 16) gate_modes<L, 1, 3, 0>(G, x, l, part);
            break;
        default:
            if constexpr (L == 32) gate_modes<L, 1, 4, 0>(G, x, l, part);
            break;
        }
        return;
    }
#define SV_ADJ2(a, b) case a * 8 + b: gate_modes<L, 2, a, b>(G, x, l, part); break;
    if constexpr (L == 8) {
        switch (G.t0 * 8 + G.t1) {
        SV_ADJ2(0, 1) SV_ADJ2(0, 2) SV_ADJ2(1, 0) SV_ADJ2(1, 2) SV_ADJ2(2, 0)
        default: gate_modes<L, 2, 2, 1>(G, x, l, part); break;
        }
    } else if constexpr (L == 16) {
        switch (G.t0 * 8 + G.t1) {
        SV_ADJ2(0, 1) SV_ADJ2(0, 2) SV_ADJ2(0, 3)
        SV_ADJ2(1, 0) SV_ADJ2(1, 2) SV_ADJ2(1, 3)
        SV_ADJ2(2, 0) SV_ADJ2(2, 1) SV_ADJ2(2, 3)
        SV_ADJ2(3, 0) SV_ADJ2(3, 1)
        default: gate_modes<L, 2, 3, 2>(G, x, l, part); break;
        }
    } else {
        switch (G.t0 * 8 + G.t1) {
        SV_ADJ2(0, 1) SV_ADJ2(0, 2) SV_ADJ2(0, 3) SV_ADJ2(0, 4)
        SV_ADJ2(1, 0) SV_ADJ2(1, 2) SV_ADJ2(1, 3) SV_ADJ2(1, 4)
        SV_ADJ2(2, 0) SV_ADJ2(2, 1) SV_ADJ2(2, 3) SV_ADJ2(2, 4)
        SV_ADJ2(3, 0) SV_ADJ2(3, 1) SV_ADJ2(3, 2) SV_ADJ2(3, 4)
        SV_ADJ2(4, 0) SV_ADJ2(4, 1) SV_ADJ2(4, 2)
        default: gate_modes<L, 2, 4, 3>(G, x, l, part); break;
        }
    }
#undef SV_ADJ2
}

template <int LB>
__global__ __launch_bounds__(256) void k_adj_block(AdjBlockLaunch a, double* part)
{
    constexpr int L = 1 << LB;
    __shared__ double acc[4][kAdjBlockMaxSlots];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < 4 * kAdjBlockMaxSlots; i += 256) (&acc[0][0])[i] = 0.0;
    __syncthreads();
    const int row = blockIdx.y;
    float2* psi = arow(a.psi, row);
    float2* lam = arow(a.lam, row);
    const int n = __builtin_ctzll(a.psi.N);
    const uint64_t ncols = 1ull << (n - LB);
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t c0 = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * 256 + wave * 64; c0 < ncols; c0 += stride) {
        const uint64_t c = c0 + lane;
        const bool live = c < ncols;
        const uint64_t base = insert_zeros(live ? c : 0, a.q, LB);
        float2 x[L], l[L];
#pragma unroll
        for (int j = 0; j < L; ++j) {
            uint64_t o = base;
#pragma unroll
            for (int i = 0; i < LB; ++i)
                if ((j >> i) & 1) o |= a.qbit[i];
            x[j] = live ? psi[o] : make_float2(0.f, 0.f);
            l[j] = live ? lam[o] : make_float2(0.f, 0.f);
        }
        for (int gi = 0; gi < a.ngates; ++gi) {
            const AdjBlockGate& G = a.gates[gi];
            double part3[3] = {0.0, 0.0, 0.0};
            dispatch_gate<L>(G, x, l, part3);
            for (int d = 0; d < G.nd; ++d) {
                const double v = wave_sum(part3[d]);
                if (lane == 0) acc[wave][G.slot[d]] += v;
            }
        }
        // recompute the addresses from an opaque copy of the base rather than
        // keeping all of them live across the gate loop
        uint64_t base2 = base;
        asm volatile("" : "+v"(base2));
        if (live) {
#pragma unroll
            for (int j = 0; j < L; ++j) {
                uint64_t o = base2;
#pragma unroll
                for (int i = 0; i < LB; ++i)
                    if ((j >> i) & 1) o |= a.qbit[i];
                psi[o] = x[j];
                lam[o] = l[j];
            }
        }
    }
    // each wave's sums (its own LDS row, written by its own lane 0)
    const uint64_t w = (uint64_t)blockIdx.x * 4 + wave;
    for (int s = lane; s < a.nslots; s += 64)
        part[((uint64_t)row * a.nslots + s) * (4ull * gridDim.x) + w] = acc[wave][s];
}

}  // namespace

int adj_block_grid(int n, int lb)
{
    const uint64_t cols = 1ull << (n - lb);
    const uint64_t want = (cols + 255) / 256;
    const uint64_t cap = (uint64_t)device_info().cu_count * 8;
    return (int)std::max<uint64_t>(1, std::min(want, cap));
}

void launch_adj_block(const AdjBlockLaunch& a, double* part, hipStream_t st)
{
    if (a.lb == 3)
        hipLaunchKernelGGL(k_adj_block<3>, dim3(a.grid, a.psi.nrows), dim3(256), 0, st, a, part);
    else if (a.lb == 4)
        hipLaunchKernelGGL(k_adj_block<4>, dim3(a.grid, a.psi.nrows), dim3(256), 0, st, a, part);
    else
        hipLaunchKernelGGL(k_adj_block<5>, dim3(a.grid, a.psi.nrows), dim3(256), 0, st, a, part);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
