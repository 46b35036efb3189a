// k_batch.hip -- many independent circuits of uneven size in ONE persistent
// launch (the batch dimension of Sec. 4.2, generalised to circuits with
// different qubit counts and gate lists).
//
// One workgroup (1024 threads) runs one circuit at a time, taking circuit
// indices from an atomic counter (circuits are sorted by size, largest
// first). The circuit's state is processed in tiles of up to 2^14
// amplitudes held in LDS (128 KiB):
//   n <= 14: the whole state is one tile. It is created in LDS as |0..0>,
//            every gate runs in LDS, and <Z_i> is reduced from LDS -- the
//            state never touches HBM.
//   n > 14:  the gate list is cut into passes; every gate of a pass acts on
//            a fixed set of 14 qubits (always including qubits 0..5, so a
//            tile is made of contiguous runs of >= 64 amplitudes). A pass
//            streams every tile of the state through LDS once and applies
//            all of its gates there. The first pass creates |0..0>, the last
//            pass reduces <Z_i> instead of writing back.
// Gate matrices are computed on the device from the parameter buffer, so a
// captured launch can be replayed with new parameters.
#include "sv_device.h"
#include "sv_internal.h"
#include "batch.h"

namespace sv {

namespace {

constexpr int kBT = 1024;

__device__ __forceinline__ float2 f2(double re, double im) { return make_float2((float)re, (float)im); }

// Gate matrix (first target = most significant index bit), complex64.
// Same definitions as the host gate math (rotations exp(-i t P / 2), OpenQASM
// U3, phase gate), evaluated in FP64 and rounded once.
__device__ int dev_gate_matrix(int kind, const double* prm, float2* m)
{
    const double h = 0.70710678118654752440;
    auto set2 = [&](float2 a, float2 b, float2 c, float2 d) { m[0] = a; m[1] = b; m[2] = c; m[3] = d; return 1; };
    const float2 z0 = f2(0, 0), o1 = f2(1, 0);
    switch (kind) {
    case SV_H: return set2(f2(h, 0), f2(h, 0), f2(h, 0), f2(-h, 0));
    case SV_X: return set2(z0, o1, o1, z0);
    case SV_Y: return set2(z0, f2(0, -1), f2(0, 1), z0);
    case SV_Z: return set2(o1, z0, z0, f2(-1, 0));
    case SV_S: return set2(o1, z0, z0, f2(0, 1));
    case SV_SDG: return set2(o1, z0, z0, f2(0, -1));
    case SV_T: return set2(o1, z0, z0, f2(h, h));
    case SV_TDG: return set2(o1, z0, z0, f2(h, -h));
    case SV_SX: return set2(f2(0.5, 0.5), f2(0.5, -0.5), f2(0.5, -0.5), f2(0.5, 0.5));
    case SV_RX: case SV_RY: case SV_RZ: {
        double s, c;
        sincos(0.5 * prm[0], &s, &c);
        if (kind == SV_RX) return set2(f2(c, 0), f2(0, -s), f2(0, -s), f2(c, 0));
        if (kind == SV_RY) return set2(f2(c, 0), f2(-s, 0), f2(s, 0), f2(c, 0));
        return set2(f2(c, -s), z0, z0, f2(c, s));
    }
    case SV_P: {
        double s, c;
        sincos(prm[0], &s, &c);
        return set2(o1, z0, z0, f2(c, s));
    }
    case SV_U3: {
        double s, c, sf, cf, sl, cl, sfl, cfl;
        sincos(0.5 * prm[0], &s, &c);
        sincos(prm[1], &sf, &cf);
        sincos(prm[2], &sl, &cl);
        sincos(prm[1] + prm[2], &sfl, &cfl);
        return set2(f2(c, 0), f2(-s * cl, -s * sl), f2(s * cf, s * sf), f2(c * cfl, c * sfl));
    }
    case SV_SWAP:
        for (int i = 0; i < 16; ++i) m[i] = z0;
        m[0] = m[15] = o1;
        m[6] = m[9] = o1;
        return 2;
    case SV_RXX: case SV_RYY: case SV_RZZ: {
        double s, c;
        sincos(0.5 * prm[0], &s, &c);
        for (int i = 0; i < 16; ++i) m[i] = z0;
        for (int i = 0; i < 4; ++i) m[i * 5] = f2(c, 0);
        if (kind == SV_RZZ) {
            // -i s Z(x)Z = diag(-is, is, is, -is)
            m[0] = f2(c, -s); m[5] = f2(c, s); m[10] = f2(c, s); m[15] = f2(c, -s);
        } else if (kind == SV_RXX) {
            // -i s X(x)X: anti-diagonal
            m[3] = m[6] = m[9] = m[12] = f2(0, -s);
        } else {
            // -i s Y(x)Y: Y(x)Y = antidiag(-1, 1, 1, -1)
            m[3] = f2(0, s); m[6] = f2(0, -s); m[9] = f2(0, -s); m[12] = f2(0, s);
        }
        return 2;
    }
    default: return 0;
    }
}

__device__ __forceinline__ uint32_t ins0(uint32_t g, const int* pos, int np)
{
    for (int i = 0; i < np; ++i) {
        const uint32_t lo = g & ((1u << pos[i]) - 1u);
        g = ((g >> pos[i]) << (pos[i] + 1)) | lo;
    }
    return g;
}

// One gate on the tile in LDS (tile-local qubit positions).
__device__ void lds_gate(float2* s, int m_bits, const BOp& op, const float2* mat)
{
    int pos[5], np = 0;
    uint32_t cmask = 0;
    pos[np++] = op.t[0];
    if (op.nt == 2) pos[np++] = op.t[1];
    for (int j = 0; j < op.nc; ++j) {
        pos[np++] = op.c[j];
        cmask |= 1u << op.c[j];
    }
    for (int i = 1; i < np; ++i)
        for (int j = i; j > 0 && pos[j - 1] > pos[j]; --j) {
            const int t = pos[j - 1];
            pos[j - 1] = pos[j];
            pos[j] = t;
        }
    const uint32_t groups = 1u << (m_bits - np);
    if (op.nt == 1) {
        const uint32_t tb = 1u << op.t[0];
        for (uint32_t g = threadIdx.x; g < groups; g += kBT) {
            const uint32_t i0 = ins0(g, pos, np) | cmask, i1 = i0 | tb;
            const float2 x0 = s[i0], x1 = s[i1];
            s[i0] = cfma(mat[1], x1, cmul(mat[0], x0));
            s[i1] = cfma(mat[3], x1, cmul(mat[2], x0));
        }
    } else {
        const uint32_t b0 = 1u << op.t[0], b1 = 1u << op.t[1];
        const uint32_t off[4] = {0u, b1, b0, b0 | b1};
        for (uint32_t g = threadIdx.x; g < groups; g += kBT) {
            const uint32_t base = ins0(g, pos, np) | cmask;
            float2 x[4], y[4];
            for (int r = 0; r < 4; ++r) x[r] = s[base | off[r]];
            for (int r = 0; r < 4; ++r) {
                float2 acc = cmul(mat[r * 4], x[0]);
                for (int c = 1; c < 4; ++c) acc = cfma(mat[r * 4 + c], x[c], acc);
                y[r] = acc;
            }
            for (int r = 0; r < 4; ++r) s[base | off[r]] = y[r];
        }
    }
}

__global__ __launch_bounds__(kBT) void k_batch(BatchArgs a)
{
    __shared__ float2 tile[1 << kTileBits];
    __shared__ int next;
    __shared__ double red[kBT / 64][kBatchMaxQubits + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(a.counter, 1);
        __syncthreads();
        const int ci = next;
        __syncthreads();
        if (ci >= a.n_circ) break;
        const BCirc c = a.circ[ci];
        const double* prm = a.params + c.param_off;
        const int m = c.m;
        const uint32_t tsize = 1u << m;
        const uint64_t ntiles = 1ull << (c.n - m);
        double zs[kBatchMaxQubits + 1];
#pragma unroll
        for (int i = 0; i <= kBatchMaxQubits; ++i) zs[i] = 0.0;
        for (int pi = c.pass_begin; pi < c.pass_end; ++pi) {
            const BPass& ps = a.pass[pi];
            const bool first = pi == c.pass_begin, last = pi == c.pass_end - 1;
            // offset of tile-local index l = tid + 1024 j: tid covers tile bits 0..9
            uint64_t off_t = 0;
            for (int b = 0; b < m && b < 10; ++b)
                if ((threadIdx.x >> b) & 1) off_t |= 1ull << ps.pos[b];
            for (uint64_t tau = 0; tau < ntiles; ++tau) {
                const uint64_t base = insert_zeros(tau, ps.pos, m);
                // fill the tile
                for (uint32_t j = 0; (j << 10) < tsize; ++j) {
                    const uint32_t l = threadIdx.x + (j << 10);
                    if (l >= tsize) break;
                    if (first) {
                        tile[l] = make_float2(base == 0 && l == 0 ? 1.f : 0.f, 0.f);
                    } else {
                        uint64_t off = off_t;
                        for (int b = 10; b < m; ++b)
                            if ((j >> (b - 10)) & 1) off |= 1ull << ps.pos[b];
                        tile[l] = a.arena[c.arena_off + base + off];
                    }
                }
                __syncthreads();
                for (int oi = ps.op_begin; oi < ps.op_end; ++oi) {
                    const BOp op = a.ops[oi];
                    double p3[3] = {0.0, 0.0, 0.0};
                    for (int q = 0; q < 3; ++q)
                        if (op.p[q] >= 0) p3[q] = prm[op.p[q]];
                    float2 mat[16];
                    dev_gate_matrix(op.kind, p3, mat);
                    lds_gate(tile, m, op, mat);
                    __syncthreads();
                }
                if (last) {
                    for (uint32_t j = 0; (j << 10) < tsize; ++j) {
                        const uint32_t l = threadIdx.x + (j << 10);
                        if (l >= tsize) break;
                        uint64_t off = off_t;
                        for (int b = 10; b < m; ++b)
                            if ((j >> (b - 10)) & 1) off |= 1ull << ps.pos[b];
                        const uint64_t gb = base + off;
                        const float2 v = tile[l];
                        const double p = (double)v.x * v.x + (double)v.y * v.y;
                        zs[kBatchMaxQubits] += p;
#pragma unroll
                        for (int i = 0; i < kBatchMaxQubits; ++i)
                            if (((gb >> i) & 1) && i < c.n) zs[i] += p;
                    }
                } else {
                    for (uint32_t j = 0; (j << 10) < tsize; ++j) {
                        const uint32_t l = threadIdx.x + (j << 10);
                        if (l >= tsize) break;
                        uint64_t off = off_t;
                        for (int b = 10; b < m; ++b)
                            if ((j >> (b - 10)) & 1) off |= 1ull << ps.pos[b];
                        a.arena[c.arena_off + base + off] = tile[l];
                    }
                }
                __syncthreads();   // tile reads/writes done before the next fill
            }
        }
        // <Z_i> = tot - 2 S_i, fixed-order reduction over the workgroup
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int i = 0; i <= kBatchMaxQubits; ++i) zs[i] += __shfl_xor(zs[i], off, 64);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i <= kBatchMaxQubits; ++i) red[wave][i] = zs[i];
        __syncthreads();
        if (threadIdx.x <= kBatchMaxQubits) {
            double t = 0.0, s = 0.0;
            for (int w = 0; w < kBT / 64; ++w) {
                t += red[w][kBatchMaxQubits];
                s += red[w][threadIdx.x];
            }
            const int i = threadIdx.x;
            if (i < SV_BATCH_OUT_STRIDE)
                a.out[(uint64_t)c.out_idx * SV_BATCH_OUT_STRIDE + i] = i < c.n ? t - 2.0 * s : 0.0;
        }
        if (threadIdx.x > kBatchMaxQubits && threadIdx.x < SV_BATCH_OUT_STRIDE)
            a.out[(uint64_t)c.out_idx * SV_BATCH_OUT_STRIDE + threadIdx.x] = 0.0;
        __syncthreads();
    }
}

__global__ void k_zero_counter(int* counter) { *counter = 0; }

}  // namespace

void launch_batch(const BatchArgs& a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, st, a.counter);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBT), 0, st, a);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
