// k_gates.hip -- plain gate sweeps: one pass over the state per gate.
//
// A gate (M, Q) with controls C updates, for every group base b (target bits
// 0, control bits 1), the 2^k amplitudes b | offset(r) in place:
// (psi[b|off(r)])_r <- M (psi[b|off(r)])_r  (Alg. 1 of Sec. 4.1.1 with the
// MoveDim done by index arithmetic instead of a tensor permute).
//
// Memory access forms, chosen per gate by the host:
//   SHFL  one target t in 1..6, no control below 7: each wave owns 128
//         consecutive amplitudes (one float4 per lane, a fully contiguous
//         1 KiB access); the pair partner lives in lane ^ 2^(t-1) of the same
//         wave and is exchanged by a cross-lane shuffle.
//   HALF  one target t >= 7, no control at qubit 0, at least 128 groups: a
//         wave takes 32 pairs of float4s; lanes 0..31 read the low members
//         (512 contiguous bytes), lanes 32..63 the high members (the same
//         bytes 2^t amplitudes on), the halves swap values by a cross-lane
//         shuffle, and every lane writes the one float4 it read. Measured
//         against a thread per pair (both members read and written by one
//         lane): 2.57-2.91 ms instead of 2.90-3.12 ms per 30-qubit sweep.
//   VEC2  no target or control is qubit 0: each member of a group is read as a
//         float4 holding two neighbouring amplitudes; consecutive lanes take
//         consecutive float4s of every member stream.
//   PAIR  one target at qubit 0: the pair (b, b|1) is one float4.
//   ODD   a control at qubit 0 (e.g. CNOT from qubit 0): float4 members as in
//         VEC2 with only the odd amplitude of each float4 updated.
//   VEC1  anything else: float2 per member.
// Accesses are non-temporal (each amplitude is touched once per sweep) when
// every written 128-byte line is written whole; otherwise cached.
// Amplitudes outside the control subspace are never read or written, except
// the even neighbours in the ODD form, which are written back unchanged.
#include <atomic>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

namespace {

enum Form { VEC1 = 1, VEC2 = 2, PAIR = 0, ODD = 3, SHFL = 4, HALF = 5 };

// HALF: threads and float4 pairs per workgroup. Two-wave workgroups, by
// default in the hardware's own order (no XCD renumbering): on a 30-qubit
// state the mean sweep over targets 7..29 took 2.595 ms against 2.642 ms
// with four-wave workgroups in XCD-contiguous order. The better order
// depends on the target (XCD-contiguous won on 7 and 21..23 there), so
// sv_sweep_order_tune can time both per target and record the choice for
// uncontrolled sweeps of that state size on that device (half_order_mask).
constexpr int kHalfBlock = 128;
constexpr int kHalfUnits = kHalfBlock / 2;

struct KGate {
    float2* p0;
    float2* p1;
    int nrow0;
    uint64_t N;
    uint64_t n_units;     // per row
    uint64_t unit0;       // first unit of this launch (launches are split at kMaxBlocks)
    uint64_t cmask;       // control bits, OR'ed into every base
    uint64_t moff[4];     // member offsets: bits of the targets selected by the member index
    int npos;             // positions where zero bits are inserted (sorted ascending)
    int pos[6];
    int t;                // SHFL: the target qubit
    int xcd;              // HALF: 1 = XCD-contiguous workgroup order, 0 = the hardware's order
    float2 m[16];         // row-major 2^k x 2^k complex64
};

__device__ __forceinline__ float2* row_ptr(float2* p0, float2* p1, int nrow0, uint64_t N, int row)
{
    return row < nrow0 ? p0 + (uint64_t)row * N : p1 + (uint64_t)(row - nrow0) * N;
}

template <int D>
__device__ __forceinline__ void matvec(const float2 (&m)[16], const float2 (&x)[D], float2 (&y)[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float2 acc = cmul(m[i * D], x[0]);
#pragma unroll
        for (int j = 1; j < D; ++j) acc = cfma(m[i * D + j], x[j], acc);
        y[i] = acc;
    }
}

template <int K, int F, int U, bool NT>
__global__ __launch_bounds__(kBlock) void k_gate(KGate a)
{
    constexpr int D = 1 << K;
    float2* psi = row_ptr(a.p0, a.p1, a.nrow0, a.N, blockIdx.y);
    float2 m[16];
#pragma unroll
    for (int i = 0; i < D * D; ++i) m[i] = a.m[i];
    const uint64_t u0 = a.unit0 + xcd_block(blockIdx.x, gridDim.x) * (kBlock * U) + threadIdx.x;

    if constexpr (F == HALF) {
        static_assert(K == 1 && U == 1, "split-halves form: one target, one pair per lane pair");
        const int lane = threadIdx.x & 63;
        const uint64_t blk = a.xcd ? xcd_block(blockIdx.x, gridDim.x) : (uint64_t)blockIdx.x;
        const uint64_t u = a.unit0 + blk * kHalfUnits + (threadIdx.x >> 6) * 32 +
                           (lane & 31);
        const bool hi = lane >= 32;
        // n_units is a multiple of 32: a wave is wholly in or out of range
        if (u < a.n_units) {
            float2* p = psi + ((insert_zeros(u << 1, a.pos, a.npos) | a.cmask) | (hi ? a.moff[1] : 0ull));
            const float4 me = ld4<NT>(p);
            float4 ot;
            ot.x = __shfl_xor(me.x, 32, 64);
            ot.y = __shfl_xor(me.y, 32, 64);
            ot.z = __shfl_xor(me.z, 32, 64);
            ot.w = __shfl_xor(me.w, 32, 64);
            // low member: y0 = m00 x0 + m01 x1; high member: y1 = m10 x0 + m11 x1
            const float2 cs = hi ? m[3] : m[0];   // coefficient of my own amplitude
            const float2 cp = hi ? m[2] : m[1];   // coefficient of the partner's
            const float2 y0 = cfma(cp, lo2(ot), cmul(cs, lo2(me)));
            const float2 y1 = cfma(cp, hi2(ot), cmul(cs, hi2(me)));
            st4<NT>(p, pack4(y0, y1));
        }
    } else if constexpr (F == VEC2 || F == ODD) {
        float4 v[U][D];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u << 1, a.pos, a.npos) | a.cmask;
            if (u < a.n_units)
#pragma unroll
                for (int j = 0; j < D; ++j) v[r][j] = ld4<NT>(psi + (base[r] | a.moff[j]));
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            float2 xl[D], xh[D], yl[D], yh[D];
#pragma unroll
            for (int j = 0; j < D; ++j) { xl[j] = lo2(v[r][j]); xh[j] = hi2(v[r][j]); }
            if constexpr (F == VEC2) matvec<D>(m, xl, yl);
            matvec<D>(m, xh, yh);
#pragma unroll
            for (int j = 0; j < D; ++j)
                st4<NT>(psi + (base[r] | a.moff[j]), pack4(F == VEC2 ? yl[j] : xl[j], yh[j]));
        }
    } else if constexpr (F == SHFL) {
        static_assert(K == 1, "shuffle form is for one target");
        const int t = a.t;
        const int lane_xor = 1 << (t - 1);
        float4 v[U];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u << 1, a.pos, a.npos) | a.cmask;
            // whole waves are in or out of range (n_units is a multiple of 64)
            if (u < a.n_units) v[r] = ld4<NT>(psi + base[r]);
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            float4 w;
            w.x = __shfl_xor(v[r].x, lane_xor, 64);
            w.y = __shfl_xor(v[r].y, lane_xor, 64);
            w.z = __shfl_xor(v[r].z, lane_xor, 64);
            w.w = __shfl_xor(v[r].w, lane_xor, 64);
            const bool hi = (base[r] >> t) & 1;
            // low member: y0 = m00 x0 + m01 x1; high member: y1 = m10 x0 + m11 x1
            const float2 cs = hi ? m[3] : m[0];   // coefficient of my own amplitude
            const float2 cp = hi ? m[2] : m[1];   // coefficient of the partner's
            const float2 y0 = cfma(cp, lo2(w), cmul(cs, lo2(v[r])));
            const float2 y1 = cfma(cp, hi2(w), cmul(cs, hi2(v[r])));
            st4<NT>(psi + base[r], pack4(y0, y1));
        }
    } else if constexpr (F == PAIR) {
        static_assert(K == 1, "pair-in-lane form is for one target");
        float4 v[U];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u, a.pos, a.npos) | a.cmask;
            if (u < a.n_units) v[r] = ld4<NT>(psi + base[r]);
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            float2 x[2] = {lo2(v[r]), hi2(v[r])}, y[2];
            matvec<2>(m, x, y);
            st4<NT>(psi + base[r], pack4(y[0], y[1]));
        }
    } else {
        float2 v[U][D];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u, a.pos, a.npos) | a.cmask;
            if (u < a.n_units)
#pragma unroll
                for (int j = 0; j < D; ++j) v[r][j] = ld2<NT>(psi + (base[r] | a.moff[j]));
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            float2 y[D];
            matvec<D>(m, v[r], y);
#pragma unroll
            for (int j = 0; j < D; ++j) st2<NT>(psi + (base[r] | a.moff[j]), y[j]);
        }
    }
}

// Diagonal gates: every amplitude of the swept subspace is multiplied by a
// phase chosen by its free-target bits. Fixed positions (controls, and the
// targets of gates that only change the all-ones pattern) are set to 1, so
// e.g. CZ touches one quarter of the state. A fixed qubit 0 is handled with
// float4 accesses that update only the odd amplitude.
struct KDiag {
    float2* p0;
    float2* p1;
    int nrow0;
    uint64_t N;
    uint64_t n_units;
    uint64_t unit0;       // first unit of this launch
    uint64_t fmask;       // fixed-to-1 bits above qubit 0
    int npos;
    int pos[5];
    int nfree;
    uint64_t fbit[2];     // free target bits, fbit[0] = most significant of the phase index
    uint64_t tmask;       // whole-state form: amplitudes without all these bits keep phase 1
    float2 ph[4];
};

__device__ __forceinline__ float2 diag_phase(const KDiag& a, uint64_t b)
{
    if ((b & a.tmask) != a.tmask) return make_float2(1.f, 0.f);
    int idx = 0;
    for (int j = 0; j < a.nfree; ++j) idx = (idx << 1) | ((b & a.fbit[j]) ? 1 : 0);
    return a.ph[idx];
}

template <int F, int U, bool NT>
__global__ __launch_bounds__(kBlock) void k_diag(KDiag a)
{
    float2* psi = row_ptr(a.p0, a.p1, a.nrow0, a.N, blockIdx.y);
    const uint64_t u0 = a.unit0 + xcd_block(blockIdx.x, gridDim.x) * (kBlock * U) + threadIdx.x;
    if constexpr (F == VEC2 || F == ODD) {
        float4 v[U];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u << 1, a.pos, a.npos) | a.fmask;
            if (u < a.n_units) v[r] = ld4<NT>(psi + base[r]);
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            const float2 y0 = F == ODD ? lo2(v[r]) : cmul(diag_phase(a, base[r]), lo2(v[r]));
            const float2 y1 = cmul(diag_phase(a, base[r] | 1), hi2(v[r]));
            st4<NT>(psi + base[r], pack4(y0, y1));
        }
    } else {
        float2 v[U];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u, a.pos, a.npos) | a.fmask;
            if (u < a.n_units) v[r] = ld2<NT>(psi + base[r]);
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            st2<NT>(psi + base[r], cmul(diag_phase(a, base[r]), v[r]));
        }
    }
}

// Every row := e_idx.
__global__ __launch_bounds__(kBlock) void k_basis(float2* p0, uint64_t N, uint64_t idx)
{
    float2* row = p0 + (uint64_t)blockIdx.y * N;
    const uint64_t n4 = N >> 1;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * kBlock) {
        float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i == (idx >> 1)) {
            if (idx & 1) z.z = 1.f;
            else z.x = 1.f;
        }
        st4(row + 2 * i, z);
    }
}

// Plain streaming copy (the bandwidth reference used to scale byte counters).
__global__ __launch_bounds__(kBlock) void k_copy(float2* __restrict__ dst, const float2* __restrict__ src, uint64_t n4)
{
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n4) st4(dst + 2 * i, ld4(src + 2 * i));
}

void sort_small(int* v, int n)
{
    for (int i = 1; i < n; ++i)
        for (int j = i; j > 0 && v[j - 1] > v[j]; --j) std::swap(v[j - 1], v[j]);
}

constexpr int kUnroll = 1;   // one unit per thread: measured best with the XCD renumbering

// A launch holds fewer than 2^32 work-items in x: sweeps of more units (states
// above 32 qubits) are split into launches of at most kMaxBlocks workgroups,
// each starting at its own first unit.
constexpr uint64_t kMaxBlocks = 1ull << 22;

template <class Args, class Launch>
void split_launch(Args a, uint64_t blocks, Launch&& launch)
{
    const uint64_t per_block = (uint64_t)kBlock * kUnroll;
    for (uint64_t b0 = 0; b0 < blocks; b0 += kMaxBlocks) {
        a.unit0 = b0 * per_block;
        launch(a, (unsigned)std::min(kMaxBlocks, blocks - b0));
        SV_HIP(hipGetLastError());
    }
}

template <int K, int F>
void dispatch_gate(const KGate& a, int rows, bool nt, hipStream_t st)
{
    const uint64_t per_block = (uint64_t)kBlock * kUnroll;
    const uint64_t blocks = (a.n_units + per_block - 1) / per_block;
    split_launch(a, blocks, [&](const KGate& x, unsigned nb) {
        if (nt)
            hipLaunchKernelGGL((k_gate<K, F, kUnroll, true>), dim3(nb, rows), dim3(kBlock), 0, st, x);
        else
            hipLaunchKernelGGL((k_gate<K, F, kUnroll, false>), dim3(nb, rows), dim3(kBlock), 0, st, x);
    });
}

void dispatch_half(const KGate& a0, int rows, bool nt, hipStream_t st)
{
    const uint64_t blocks = a0.n_units / kHalfUnits;
    for (uint64_t b0 = 0; b0 < blocks; b0 += kMaxBlocks) {
        KGate a = a0;
        a.unit0 = b0 * kHalfUnits;
        const unsigned nb = (unsigned)std::min(kMaxBlocks, blocks - b0);
        if (nt)
            hipLaunchKernelGGL((k_gate<1, HALF, 1, true>), dim3(nb, rows), dim3(kHalfBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_gate<1, HALF, 1, false>), dim3(nb, rows), dim3(kHalfBlock), 0, st, a);
        SV_HIP(hipGetLastError());
    }
}

// Per device and state size: bit t set = uncontrolled split-halves sweeps on
// target t take the XCD-contiguous workgroup order. Only the launch order
// depends on it; every pair is computed by the same instructions.
constexpr int kOrderDevices = 64;
std::atomic<uint64_t> g_half_order[kOrderDevices][64];

}  // namespace

uint64_t half_order_mask(int n)
{
    const int dev = device_info().device;
    if (dev < 0 || dev >= kOrderDevices || n < 0 || n >= 64) return 0;
    return g_half_order[dev][n].load(std::memory_order_relaxed);
}

void set_half_order_mask(int n, uint64_t mask)
{
    const int dev = device_info().device;
    if (dev < 0 || dev >= kOrderDevices || n < 0 || n >= 64) return;
    g_half_order[dev][n].store(mask, std::memory_order_relaxed);
}

bool half_sweep_applies(int n, int t)
{
    return n >= 8 && t >= 7 && t < n;
}

void launch_half_identity(const Rows& rows, int t, bool xcd, hipStream_t st)
{
    const int n = __builtin_ctzll(rows.N);
    KGate a{};
    a.p0 = rows.p0;
    a.p1 = rows.p1;
    a.nrow0 = rows.nrow0;
    a.N = rows.N;
    a.m[0] = make_float2(1.0f, 0.0f);
    a.m[1] = make_float2(0.0f, 0.0f);
    a.m[2] = make_float2(0.0f, 0.0f);
    a.m[3] = make_float2(1.0f, 0.0f);
    a.moff[0] = 0;
    a.moff[1] = 1ull << t;
    a.pos[a.npos++] = t;
    a.n_units = 1ull << (n - 2);                  // float4 pairs of the whole state
    a.xcd = xcd ? 1 : 0;
    dispatch_half(a, rows.nrows, t >= kFullLineQubit, st);
}

void launch_gate(const GateLaunch& g, hipStream_t st)
{
    const int n = __builtin_ctzll(g.rows.N);
    KGate a{};
    a.p0 = g.rows.p0;
    a.p1 = g.rows.p1;
    a.nrow0 = g.rows.nrow0;
    a.N = g.rows.N;
    const int D = 1 << g.k;
    for (int i = 0; i < D * D; ++i) a.m[i] = g.m[i];
    for (int r = 0; r < D; ++r) {
        uint64_t off = 0;
        for (int j = 0; j < g.k; ++j)
            if ((r >> (g.k - 1 - j)) & 1) off |= 1ull << g.targets[j];
        a.moff[r] = off;
    }
    int lowest_t = 64, lowest_c = 64;
    for (int j = 0; j < g.k; ++j) lowest_t = std::min(lowest_t, g.targets[j]);
    for (int j = 0; j < g.nc; ++j) lowest_c = std::min(lowest_c, g.controls[j]);
    const int rows = g.rows.nrows;
    const uint64_t groups = 1ull << (n - g.k - g.nc);

    // SHFL: one target in 1..6, every control >= 7, whole waves of 128 amplitudes
    if (g.k == 1 && lowest_t >= 1 && lowest_t <= 6 && lowest_c >= 7 && n - g.nc >= 7) {
        for (int j = 0; j < g.nc; ++j) {
            a.pos[a.npos++] = g.controls[j];
            a.cmask |= 1ull << g.controls[j];
        }
        sort_small(a.pos, a.npos);
        a.t = g.targets[0];
        a.n_units = 1ull << (n - g.nc - 1);      // float4s in the control subspace
        dispatch_gate<1, SHFL>(a, rows, true, st);
        return;
    }
    // insert positions: targets and controls, except a control at qubit 0 in
    // the ODD form (there the float4 spans bit 0 and only the odd half changes)
    const bool odd = lowest_c == 0 && lowest_t >= 1;
    for (int j = 0; j < g.k; ++j) a.pos[a.npos++] = g.targets[j];
    for (int j = 0; j < g.nc; ++j) {
        a.cmask |= 1ull << g.controls[j];
        if (!(odd && g.controls[j] == 0)) a.pos[a.npos++] = g.controls[j];
    }
    sort_small(a.pos, a.npos);
    // whole 128-byte lines are written when no target/control sits below
    // qubit 4 (a control at qubit 0 in the ODD form still writes both halves)
    const bool nt = a.npos == 0 || a.pos[0] >= kFullLineQubit;
    if (odd) {
        a.cmask &= ~1ull;
        a.n_units = groups;                      // one float4 (two amplitudes, bit 0 free) per group member
        if (g.k == 1) dispatch_gate<1, ODD>(a, rows, nt, st);
        else dispatch_gate<2, ODD>(a, rows, nt, st);
    } else if (g.k == 1 && lowest_t >= 7 && lowest_c >= 1 && groups >= 2 * kHalfUnits) {
        a.n_units = groups >> 1;                 // float4 pairs: a power of two >= 128
        a.xcd = g.nc == 0 ? (int)((half_order_mask(n) >> g.targets[0]) & 1) : 0;
        dispatch_half(a, rows, nt, st);
    } else if (std::min(lowest_t, lowest_c) >= 1 && groups >= 2) {
        a.n_units = groups >> 1;
        if (g.k == 1) dispatch_gate<1, VEC2>(a, rows, nt, st);
        else dispatch_gate<2, VEC2>(a, rows, nt, st);
    } else if (g.k == 1 && g.targets[0] == 0) {
        // pair (b, b|1) in one float4: the zero inserted at bit 0 is the target
        a.n_units = groups;
        // the inserted zero at bit 0 lies inside the float4: only controls split lines
        dispatch_gate<1, PAIR>(a, rows, lowest_c >= kFullLineQubit, st);
    } else {
        a.n_units = groups;
        if (g.k == 1) dispatch_gate<1, VEC1>(a, rows, nt, st);
        else dispatch_gate<2, VEC1>(a, rows, nt, st);
    }
}

void launch_diag(const DiagLaunch& d, hipStream_t st)
{
    const int n = __builtin_ctzll(d.rows.N);
    KDiag a{};
    a.p0 = d.rows.p0;
    a.p1 = d.rows.p1;
    a.nrow0 = d.rows.nrow0;
    a.N = d.rows.N;
    bool fixed0 = false;
    for (int j = 0; j < d.nfixed; ++j) {
        if (d.fixed[j] == 0) {
            fixed0 = true;
            continue;
        }
        a.pos[a.npos++] = d.fixed[j];
        a.fmask |= 1ull << d.fixed[j];
    }
    sort_small(a.pos, a.npos);
    a.nfree = d.nfree;
    for (int j = 0; j < d.nfree; ++j) a.fbit[j] = 1ull << d.freeq[j];
    for (int i = 0; i < (1 << d.nfree); ++i) a.ph[i] = d.ph[i];
    // every fixed qubit below 4 (e.g. CZ on two of qubits 0..3): every
    // 128-byte line holds changed amplitudes, so the sweep covers the whole
    // state in whole lines (non-temporal), leaving the amplitudes outside the
    // fixed pattern at phase 1 (measured 2.6 ms instead of 3.1-3.3 ms for
    // CZ(0,1), CZ(1,2) at 30 qubits; with fixed qubits >= 4 too -- half or
    // fewer of the lines touched -- the subspace sweep is as fast)
    if (d.nfixed > 0 && (a.npos == 0 || a.pos[a.npos - 1] < kFullLineQubit) && n >= 8) {
        for (int j = 0; j < d.nfixed; ++j) a.tmask |= 1ull << d.fixed[j];
        a.npos = 0;
        a.fmask = 0;
        a.n_units = 1ull << (n - 1);
        const uint64_t per_block = (uint64_t)kBlock * kUnroll;
        const uint64_t blocks = (a.n_units + per_block - 1) / per_block;
        const int rows = d.rows.nrows;
        split_launch(a, blocks, [&](const KDiag& x, unsigned nb) {
            hipLaunchKernelGGL((k_diag<VEC2, kUnroll, true>), dim3(nb, rows), dim3(kBlock), 0, st, x);
        });
        return;
    }
    const uint64_t per_block = (uint64_t)kBlock * kUnroll;
    const int rows = d.rows.nrows;
    // amplitudes in the swept subspace, counting bit 0 as free: fixed
    // positions lie in 1..n-1, so there are at least two and the float4 forms
    // always apply
    a.n_units = 1ull << (n - a.npos - 1);
    const uint64_t blocks = (a.n_units + per_block - 1) / per_block;
    const bool nt = a.npos == 0 || a.pos[0] >= kFullLineQubit;
    split_launch(a, blocks, [&](const KDiag& x, unsigned nb) {
        if (fixed0 && nt)
            hipLaunchKernelGGL((k_diag<ODD, kUnroll, true>), dim3(nb, rows), dim3(kBlock), 0, st, x);
        else if (fixed0)
            hipLaunchKernelGGL((k_diag<ODD, kUnroll, false>), dim3(nb, rows), dim3(kBlock), 0, st, x);
        else if (nt)
            hipLaunchKernelGGL((k_diag<VEC2, kUnroll, true>), dim3(nb, rows), dim3(kBlock), 0, st, x);
        else
            hipLaunchKernelGGL((k_diag<VEC2, kUnroll, false>), dim3(nb, rows), dim3(kBlock), 0, st, x);
    });
}

void launch_basis(const Rows& r, uint64_t idx, hipStream_t st)
{
    // rows hold N >= 2 amplitudes (n >= 1), a whole number of float4s
    const uint64_t n4 = r.N >> 1;
    const uint64_t blocks = std::min<uint64_t>((n4 + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(k_basis, dim3((unsigned)blocks, r.nrows), dim3(kBlock), 0, st, r.p0, r.N, idx);
    SV_HIP(hipGetLastError());
}

void launch_copy(void* dst, const void* src, uint64_t bytes, hipStream_t st)
{
    const uint64_t n4 = bytes / 16;
    // at most kMaxBlocks workgroups per launch
    const uint64_t chunk = kMaxBlocks * kBlock;
    for (uint64_t i0 = 0; i0 < n4; i0 += chunk) {
        const uint64_t m = std::min(chunk, n4 - i0);
        hipLaunchKernelGGL(k_copy, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           static_cast<float2*>(dst) + 2 * i0, static_cast<const float2*>(src) + 2 * i0, m);
        SV_HIP(hipGetLastError());
    }
}

}  // namespace sv
