// k_batch.hip -- many independent circuits of uneven size in ONE persistent
// launch (the batch dimension of Sec. 4.2, generalised to circuits with
// different qubit counts and gate lists), captured in a hipGraph together
// with a small prologue kernel.
//
// Prologue (one thread per gate): every gate matrix of every circuit is
// computed once from the parameter block (so a replay of the graph reads new
// parameters), and the queue and pass counters are cleared.
//
// Persistent kernel: each workgroup (NT = 256, 512 or 1024 threads) takes
// tasks from an atomic counter. A task is one tile of one pass of one
// circuit; a tile holds up to 2^T amplitudes in LDS (T = 10..14, the plan's
// tile width; 2^14 complex64 = 128 KiB), sized at launch as dynamic LDS.
//   n <= T:  the whole circuit is one task: the state is created in LDS as
//            |0..0>, every gate runs in LDS, <Z_i> is reduced from LDS -- the
//            state never touches HBM.
//   n > T:   the gate list is cut into passes whose gates all act inside one
//            T-qubit tile (always including the lowest qubits, so a tile is
//            made of contiguous runs of >= 32 amplitudes); the 2^(n-T) tiles
//            of a pass are independent tasks, spread over many workgroups. A tile
//            of pass p waits (bounded) until every tile of pass p-1 of its
//            circuit is done; tasks are ordered so such a wait only ever
//            depends on tasks handed out earlier. The first pass creates
//            |0..0>; the last pass reduces <Z_i> per tile, and the workgroup
//            that finishes the last tile sums the tiles' partials in tile
//            order (deterministic).
#include "batch.h"
#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

namespace {

constexpr int kZ = kBatchMaxQubits + 1;

__device__ __forceinline__ float2 f2(double re, double im) { return make_float2((float)re, (float)im); }

// Gate matrix (first target = most significant index bit), complex64. The
// same definitions as the host gate math (rotations exp(-i t P / 2),
// OpenQASM U3, phase gate), evaluated in FP64 and rounded once.
__device__ void dev_gate_matrix(int kind, const double* prm, float2* m)
{
    const double h = 0.70710678118654752440;
    const float2 z0 = f2(0, 0), o1 = f2(1, 0);
    for (int i = 0; i < kMatStride; ++i) m[i] = z0;
    auto set2 = [&](float2 a, float2 b, float2 c, float2 d) { m[0] = a; m[1] = b; m[2] = c; m[3] = d; };
    switch (kind) {
    case SV_H: set2(f2(h, 0), f2(h, 0), f2(h, 0), f2(-h, 0)); break;
    case SV_X: set2(z0, o1, o1, z0); break;
    case SV_Y: set2(z0, f2(0, -1), f2(0, 1), z0); break;
    case SV_Z: set2(o1, z0, z0, f2(-1, 0)); break;
    case SV_S: set2(o1, z0, z0, f2(0, 1)); break;
    case SV_SDG: set2(o1, z0, z0, f2(0, -1)); break;
    case SV_T: set2(o1, z0, z0, f2(h, h)); break;
    case SV_TDG: set2(o1, z0, z0, f2(h, -h)); break;
    case SV_SX: set2(f2(0.5, 0.5), f2(0.5, -0.5), f2(0.5, -0.5), f2(0.5, 0.5)); break;
    case SV_RX: case SV_RY: case SV_RZ: {
        double s, c;
        sincos(0.5 * prm[0], &s, &c);
        if (kind == SV_RX) set2(f2(c, 0), f2(0, -s), f2(0, -s), f2(c, 0));
        else if (kind == SV_RY) set2(f2(c, 0), f2(-s, 0), f2(s, 0), f2(c, 0));
        else set2(f2(c, -s), z0, z0, f2(c, s));
        break;
    }
    case SV_P: {
        double s, c;
        sincos(prm[0], &s, &c);
        set2(o1, z0, z0, f2(c, s));
        break;
    }
    case SV_U3: {
        double s, c, sf, cf, sl, cl, sfl, cfl;
        sincos(0.5 * prm[0], &s, &c);
        sincos(prm[1], &sf, &cf);
        sincos(prm[2], &sl, &cl);
        sincos(prm[1] + prm[2], &sfl, &cfl);
        set2(f2(c, 0), f2(-s * cl, -s * sl), f2(s * cf, s * sf), f2(c * cfl, c * sfl));
        break;
    }
    case SV_SWAP:
        m[0] = m[15] = o1;
        m[6] = m[9] = o1;
        break;
    case SV_RXX: case SV_RYY: case SV_RZZ: {
        double s, c;
        sincos(0.5 * prm[0], &s, &c);
        for (int i = 0; i < 4; ++i) m[i * 5] = f2(c, 0);
        if (kind == SV_RZZ) {
            // cos I - i sin Z(x)Z, Z(x)Z = diag(1, -1, -1, 1)
            m[0] = f2(c, -s); m[5] = f2(c, s); m[10] = f2(c, s); m[15] = f2(c, -s);
        } else if (kind == SV_RXX) {
            // X(x)X = antidiag(1, 1, 1, 1)
            m[3] = m[6] = m[9] = m[12] = f2(0, -s);
        } else {
            // Y(x)Y = antidiag(-1, 1, 1, -1)
            m[3] = f2(0, s); m[6] = f2(0, -s); m[9] = f2(0, -s); m[12] = f2(0, s);
        }
        break;
    }
    default: break;
    }
}

__global__ __launch_bounds__(256) void k_batch_prep(BatchArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < a.n_ops) {
        const BOp op = a.ops[i];
        double prm[3];
        for (int q = 0; q < 3; ++q) prm[q] = op.p[q] >= 0 ? a.params[op.p[q]] : 0.0;
        float2 m[kMatStride];
        dev_gate_matrix(op.kind, prm, m);
        for (int q = 0; q < kMatStride; ++q) a.mats[(size_t)i * kMatStride + q] = m[q];
    }
    if (i < a.n_pass) a.done[i] = 0;
    if (i == 0) *a.counter = 0;
}

__device__ __forceinline__ uint32_t ins0(uint32_t g, const int* pos, int np)
{
    for (int i = 0; i < np; ++i) {
        const uint32_t lo = g & ((1u << pos[i]) - 1u);
        g = ((g >> pos[i]) << (pos[i] + 1)) | lo;
    }
    return g;
}

// One gate on the tile in LDS.
template <int NT>
__device__ __forceinline__ void lds_gate(float2* s, int m_bits, const BOp& op, const float2* __restrict__ mat)
{
    const uint32_t groups = 1u << (m_bits - op.np);
    if (op.nt == 1) {
        const float2 m0 = mat[0], m1 = mat[1], m2 = mat[2], m3 = mat[3];
        const uint32_t tb = op.off[1];
        for (uint32_t g = threadIdx.x; g < groups; g += NT) {
            const uint32_t i0 = ins0(g, op.pos, op.np) | op.cmask, i1 = i0 | tb;
            const float2 x0 = s[i0], x1 = s[i1];
            s[i0] = cfma(m1, x1, cmul(m0, x0));
            s[i1] = cfma(m3, x1, cmul(m2, x0));
        }
    } else {
        float2 mm[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) mm[q] = mat[q];
        for (uint32_t g = threadIdx.x; g < groups; g += NT) {
            const uint32_t base = ins0(g, op.pos, op.np) | op.cmask;
            float2 x[4], y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = s[base | op.off[r]];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float2 acc = cmul(mm[r * 4], x[0]);
#pragma unroll
                for (int c = 1; c < 4; ++c) acc = cfma(mm[r * 4 + c], x[c], acc);
                y[r] = acc;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) s[base | op.off[r]] = y[r];
        }
    }
}

// ---------------------------------------------------------- register phases
//
// Thread t (t < 2^(m-4)) holds the 16 amplitudes whose tile index has the
// bits of t on the phase's complement positions and every combination j on
// its four qubits g[0..3] (bit i of j <-> qubit g[i]). Gates of the phase act
// on those four qubits only, so they run in registers; the tile goes through
// LDS once per phase instead of once per gate.

template <int P>
__device__ __forceinline__ void rg1(float2 (&v)[16], const float2* __restrict__ mat, int cm)
{
    const float2 m0 = mat[0], m1 = mat[1], m2 = mat[2], m3 = mat[3];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j & (1 << P)) continue;
        if ((j & cm) != cm) continue;
        const int j1 = j | (1 << P);
        const float2 x0 = v[j], x1 = v[j1];
        v[j] = cfma(m1, x1, cmul(m0, x0));
        v[j1] = cfma(m3, x1, cmul(m2, x0));
    }
}

// two targets: P0 is the most significant bit of the 4x4 matrix index
template <int P0, int P1>
__device__ __forceinline__ void rg2(float2 (&v)[16], const float2* __restrict__ mat, int cm)
{
    float2 mm[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) mm[q] = mat[q];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j & ((1 << P0) | (1 << P1))) continue;
        if ((j & cm) != cm) continue;
        const int o[4] = {j, j | (1 << P1), j | (1 << P0), j | (1 << P0) | (1 << P1)};
        float2 x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = v[o[r]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float2 acc = cmul(mm[r * 4], x[0]);
#pragma unroll
            for (int c = 1; c < 4; ++c) acc = cfma(mm[r * 4 + c], x[c], acc);
            v[o[r]] = acc;
        }
    }
}

__device__ __forceinline__ void reg_gate(float2 (&v)[16], const BOp& op, const float2* __restrict__ mat)
{
    if (op.nt == 1) {
        switch (op.rt[0]) {
        case 0: rg1<0>(v, mat, op.rcmask); break;
        case 1: rg1<1>(v, mat, op.rcmask); break;
        case 2: rg1<2>(v, mat, op.rcmask); break;
        default: rg1<3>(v, mat, op.rcmask); break;
        }
        return;
    }
    switch (op.rt[0] * 4 + op.rt[1]) {
    case 1: rg2<0, 1>(v, mat, op.rcmask); break;
    case 2: rg2<0, 2>(v, mat, op.rcmask); break;
    case 3: rg2<0, 3>(v, mat, op.rcmask); break;
    case 4: rg2<1, 0>(v, mat, op.rcmask); break;
    case 6: rg2<1, 2>(v, mat, op.rcmask); break;
    case 7: rg2<1, 3>(v, mat, op.rcmask); break;
    case 8: rg2<2, 0>(v, mat, op.rcmask); break;
    case 9: rg2<2, 1>(v, mat, op.rcmask); break;
    case 11: rg2<2, 3>(v, mat, op.rcmask); break;
    case 12: rg2<3, 0>(v, mat, op.rcmask); break;
    case 13: rg2<3, 1>(v, mat, op.rcmask); break;
    default: rg2<3, 2>(v, mat, op.rcmask); break;
    }
}

// One pass on the tile in LDS as register phases. A unit u < 2^(m-4) is the
// set of 16 amplitudes that share the complement bits u; the units of a phase
// are disjoint, so the threads take them in any order.
template <int NT>
__device__ void run_phases(float2* tile, int m, const BPass& ps, const BatchArgs& a)
{
    const uint32_t units = 1u << (m - kRegBits);
    for (int hi = ps.phase_begin; hi < ps.phase_end; ++hi) {
        const BPhase ph = a.phases[hi];
        if (ph.g[0] < 0) {
            // a gate on more than four qubits: one LDS sweep
            for (int oi = ph.op_begin; oi < ph.op_end; ++oi) {
                lds_gate<NT>(tile, m, a.ops[oi], a.mats + (size_t)oi * kMatStride);
                __syncthreads();
            }
            continue;
        }
        uint32_t goff[kRegBits];
        uint32_t gmask = 0;
#pragma unroll
        for (int i = 0; i < kRegBits; ++i) {
            goff[i] = 1u << ph.g[i];
            gmask |= goff[i];
        }
        for (uint32_t u = threadIdx.x; u < units; u += NT) {
            // deposit the unit index on the complement positions
            uint32_t base = 0;
            for (int b = 0, k = 0; b < m; ++b) {
                if ((gmask >> b) & 1) continue;
                if ((u >> k) & 1) base |= 1u << b;
                ++k;
            }
            float2 v[16];
            uint32_t off[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                uint32_t o = base;
#pragma unroll
                for (int i = 0; i < kRegBits; ++i)
                    if ((j >> i) & 1) o |= goff[i];
                off[j] = o;
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = tile[off[j]];
            for (int oi = ph.op_begin; oi < ph.op_end; ++oi) reg_gate(v, a.ops[oi], a.mats + (size_t)oi * kMatStride);
            // each unit writes back exactly the amplitudes it read
#pragma unroll
            for (int j = 0; j < 16; ++j) tile[off[j]] = v[j];
        }
        __syncthreads();
    }
}

// Offset inside the state of tile-local index l = threadIdx.x + NT j: the
// thread's own bits (off_t) plus the bits of j on tile positions LB.. (LB =
// log2 NT).
template <int LB>
__device__ __forceinline__ uint64_t tile_off(const int* pos, int m, uint64_t off_t, uint32_t j)
{
    uint64_t off = off_t;
    for (int b = LB; b < m; ++b)
        if ((j >> (b - LB)) & 1) off |= 1ull << pos[b];
    return off;
}

template <int NT>
__device__ __forceinline__ void wg_sum(double (&zs)[kZ], double (*red)[kZ])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int i = 0; i < kZ; ++i) zs[i] += __shfl_xor(zs[i], off, 64);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < kZ; ++i) red[wave][i] = zs[i];
    __syncthreads();
}

constexpr int log2i(int x) { return x <= 1 ? 0 : 1 + log2i(x / 2); }

template <int NT>
__global__ __launch_bounds__(NT) void k_batch(BatchArgs a)
{
    constexpr int LB = log2i(NT);
    constexpr int NW = NT / 64;
    extern __shared__ float2 tile[];         // 2^m complex64, m <= the plan's tile width
    __shared__ double red[NW][kZ];
    __shared__ int s_pos[kMaxTileBits];      // the pass's tile qubits (LDS: indexed at run time)
    __shared__ int s_task, s_final, s_late;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(a.counter, 1);
        __syncthreads();
        const int ti = s_task;
        __syncthreads();
        if (ti >= a.n_tasks) break;
        const BTask tk = a.tasks[ti];
        const BCirc c = a.circ[tk.circ];
        const BPass& ps = a.pass[tk.pass];
        const int m = c.m;
        if (threadIdx.x < kMaxTileBits) s_pos[threadIdx.x] = ps.pos[threadIdx.x];
        const uint32_t tsize = 1u << m;
        const bool first = tk.pass == c.pass_begin, last = tk.pass == c.pass_end - 1;
        if (threadIdx.x == 0) {
            s_late = 0;
            if (!first) {
                // every tile of the previous pass (handed out earlier) must be done
                int it = 0;
                while (__hip_atomic_load(a.done + tk.pass - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < c.ntiles) {
                    __builtin_amdgcn_s_sleep(4);
                    if (++it > (1 << 24)) {
                        s_late = 1;    // give up: the circuit's output becomes NaN
                        break;
                    }
                }
                __threadfence();
            }
        }
        __syncthreads();
        const uint64_t base = insert_zeros((uint64_t)tk.tile, s_pos, m);
        uint64_t off_t = 0;
        for (int b = 0; b < m && b < LB; ++b)
            if ((threadIdx.x >> b) & 1) off_t |= 1ull << s_pos[b];
        // fill the tile
        for (uint32_t j = 0; (j << LB) < tsize; ++j) {
            const uint32_t l = threadIdx.x + (j << LB);
            if (l >= tsize) break;
            if (first) tile[l] = make_float2(base == 0 && l == 0 ? 1.f : 0.f, 0.f);
            else tile[l] = ld2<false>(a.arena + c.arena_off + base + tile_off<LB>(s_pos, m, off_t, j));
        }
        __syncthreads();
        if (ps.phase_end > ps.phase_begin) {
            run_phases<NT>(tile, m, ps, a);
        } else {
            for (int oi = ps.op_begin; oi < ps.op_end; ++oi) {
                lds_gate<NT>(tile, m, a.ops[oi], a.mats + (size_t)oi * kMatStride);
                __syncthreads();
            }
        }
        if (last) {
            double zs[kZ];
#pragma unroll
            for (int i = 0; i < kZ; ++i) zs[i] = 0.0;
            for (uint32_t j = 0; (j << LB) < tsize; ++j) {
                const uint32_t l = threadIdx.x + (j << LB);
                if (l >= tsize) break;
                const uint64_t gb = base + tile_off<LB>(s_pos, m, off_t, j);
                const float2 v = tile[l];
                const double p = (double)v.x * v.x + (double)v.y * v.y;
                zs[kBatchMaxQubits] += p;
#pragma unroll
                for (int i = 0; i < kBatchMaxQubits; ++i)
                    if ((gb >> i) & 1) zs[i] += p;
            }
            wg_sum<NT>(zs, red);
            if (c.ntiles == 1) {
                if (threadIdx.x < SV_BATCH_OUT_STRIDE) {
                    const int i = threadIdx.x;
                    double t = 0.0, s = 0.0;
                    if (i < c.n)
                        for (int w = 0; w < NW; ++w) {
                            t += red[w][kBatchMaxQubits];
                            s += red[w][i];
                        }
                    a.out[(size_t)c.out_idx * SV_BATCH_OUT_STRIDE + i] =
                        s_late ? __builtin_nan("") : (i < c.n ? t - 2.0 * s : 0.0);
                }
            } else if (threadIdx.x < kZ) {
                double s = 0.0;
                for (int w = 0; w < NW; ++w) s += red[w][threadIdx.x];
                a.zpart[(size_t)(c.zpart_off + tk.tile) * kZ + threadIdx.x] = s_late ? __builtin_nan("") : s;
            }
        } else {
            for (uint32_t j = 0; (j << LB) < tsize; ++j) {
                const uint32_t l = threadIdx.x + (j << LB);
                if (l >= tsize) break;
                st2<false>(a.arena + c.arena_off + base + tile_off<LB>(s_pos, m, off_t, j), tile[l]);
            }
        }
        __syncthreads();   // all results written before the pass counter moves
        if (threadIdx.x == 0) {
            s_final = 0;
            if (c.ntiles > 1) {
                __threadfence();
                const int old = atomicAdd(a.done + tk.pass, 1);
                if (last && old == c.ntiles - 1) {
                    s_final = 1;
                    __threadfence();
                }
            }
        }
        __syncthreads();
        if (s_final && threadIdx.x < SV_BATCH_OUT_STRIDE) {
            // every tile's partial is in: sum them in tile order
            const int i = threadIdx.x;
            double t = 0.0, s = 0.0;
            if (i < c.n)
                for (int q = 0; q < c.ntiles; ++q) {
                    const double* zp = a.zpart + (size_t)(c.zpart_off + q) * kZ;
                    t += zp[kBatchMaxQubits];
                    s += zp[i];
                }
            a.out[(size_t)c.out_idx * SV_BATCH_OUT_STRIDE + i] = i < c.n ? t - 2.0 * s : 0.0;
        }
        __syncthreads();
    }
}

template <int NT>
void* batch_kernel()
{
    return reinterpret_cast<void*>(&k_batch<NT>);
}

}  // namespace

size_t batch_lds_bytes(int tile_bits)
{
    return (sizeof(float2) << tile_bits);
}

int batch_max_wg_per_cu(int threads, int tile_bits)
{
    int nb = 0;
    const size_t lds = batch_lds_bytes(tile_bits);
    void* f = threads == 256 ? batch_kernel<256>() : threads == 512 ? batch_kernel<512>() : batch_kernel<1024>();
    SV_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    SV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, threads, lds));
    return std::max(nb, 1);
}

void launch_batch(const BatchArgs& a, int grid, int threads, int tile_bits, hipStream_t st)
{
    const int items = std::max(std::max(a.n_ops, a.n_pass), 1);
    hipLaunchKernelGGL(k_batch_prep, dim3((items + 255) / 256), dim3(256), 0, st, a);
    SV_HIP(hipGetLastError());
    const size_t lds = batch_lds_bytes(tile_bits);
    switch (threads) {
    case 256: hipLaunchKernelGGL(k_batch<256>, dim3(grid), dim3(256), lds, st, a); break;
    case 512: hipLaunchKernelGGL(k_batch<512>, dim3(grid), dim3(512), lds, st, a); break;
    default: hipLaunchKernelGGL(k_batch<1024>, dim3(grid), dim3(1024), lds, st, a); break;
    }
    SV_HIP(hipGetLastError());
}

}  // namespace sv
