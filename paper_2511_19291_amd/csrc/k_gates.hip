// k_gates.hip -- plain gate sweeps: one pass over the state per gate.
//
// A gate (M, Q) with controls C updates, for every group base b (target bits
// 0, control bits 1), the 2^k amplitudes b | offset(r) in place:
// (psi[b|off(r)])_r <- M (psi[b|off(r)])_r  (Alg. 1 of Sec. 4.1.1 with the
// MoveDim done by index arithmetic instead of a tensor permute).
//
// Memory access: consecutive threads take consecutive group bases, so every
// member stream is read and written with coalesced 16-byte (float4) accesses
// whenever no target or control is qubit 0 (two neighbouring amplitudes then
// belong to the same member). A gate on qubit 0 alone keeps the pair inside
// one float4. Other qubit-0 cases use 8-byte accesses. Amplitudes outside the
// control subspace are never touched.
#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

namespace {

struct KGate {
    float2* p0;
    float2* p1;
    int nrow0;
    uint64_t N;
    uint64_t n_units;     // per row
    uint64_t cmask;       // control bits, OR'ed into every base
    uint64_t moff[4];     // member offsets: bits of the targets selected by the member index
    int npos;             // positions where zero bits are inserted (sorted ascending)
    int pos[6];
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

// VEC = 2: each member access is a float4 holding two neighbouring
//          amplitudes (requires every target/control >= 1).
// VEC = 1: float2 per member.
// VEC = 0: k = 1 with target 0: one float4 holds the whole pair.
template <int K, int VEC, int U>
__global__ __launch_bounds__(kBlock) void k_gate(KGate a)
{
    constexpr int D = 1 << K;
    float2* psi = row_ptr(a.p0, a.p1, a.nrow0, a.N, blockIdx.y);
    float2 m[16];
#pragma unroll
    for (int i = 0; i < D * D; ++i) m[i] = a.m[i];
    const uint64_t u0 = (uint64_t)blockIdx.x * (kBlock * U) + threadIdx.x;

    if constexpr (VEC == 2) {
        float4 v[U][D];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u << 1, a.pos, a.npos) | a.cmask;
            if (u < a.n_units)
#pragma unroll
                for (int j = 0; j < D; ++j) v[r][j] = *reinterpret_cast<const float4*>(psi + (base[r] | a.moff[j]));
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            float2 xl[D], xh[D], yl[D], yh[D];
#pragma unroll
            for (int j = 0; j < D; ++j) { xl[j] = lo2(v[r][j]); xh[j] = hi2(v[r][j]); }
            matvec<D>(m, xl, yl);
            matvec<D>(m, xh, yh);
#pragma unroll
            for (int j = 0; j < D; ++j)
                *reinterpret_cast<float4*>(psi + (base[r] | a.moff[j])) = pack4(yl[j], yh[j]);
        }
    } else if constexpr (VEC == 0) {
        static_assert(K == 1, "pair-in-lane form is for one target");
        float4 v[U];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u, a.pos, a.npos) | a.cmask;
            if (u < a.n_units) v[r] = *reinterpret_cast<const float4*>(psi + base[r]);
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            float2 x[2] = {lo2(v[r]), hi2(v[r])}, y[2];
            matvec<2>(m, x, y);
            *reinterpret_cast<float4*>(psi + base[r]) = pack4(y[0], y[1]);
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
                for (int j = 0; j < D; ++j) v[r][j] = psi[base[r] | a.moff[j]];
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            float2 y[D];
            matvec<D>(m, v[r], y);
#pragma unroll
            for (int j = 0; j < D; ++j) psi[base[r] | a.moff[j]] = y[j];
        }
    }
}

// Diagonal gates: every amplitude of the swept subspace is multiplied by a
// phase chosen by its free-target bits. Fixed positions (controls, and the
// targets of gates that only change the all-ones pattern) are set to 1, so
// e.g. CZ touches one quarter of the state.
struct KDiag {
    float2* p0;
    float2* p1;
    int nrow0;
    uint64_t N;
    uint64_t n_units;
    uint64_t fmask;       // fixed-to-1 bits
    int npos;
    int pos[5];
    int nfree;
    uint64_t fbit[2];     // free target bits, fbit[0] = most significant of the phase index
    float2 ph[4];
};

__device__ __forceinline__ float2 diag_phase(const KDiag& a, uint64_t b)
{
    int idx = 0;
    for (int j = 0; j < a.nfree; ++j) idx = (idx << 1) | ((b & a.fbit[j]) ? 1 : 0);
    return a.ph[idx];
}

template <int VEC, int U>
__global__ __launch_bounds__(kBlock) void k_diag(KDiag a)
{
    float2* psi = row_ptr(a.p0, a.p1, a.nrow0, a.N, blockIdx.y);
    const uint64_t u0 = (uint64_t)blockIdx.x * (kBlock * U) + threadIdx.x;
    if constexpr (VEC == 2) {
        float4 v[U];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u << 1, a.pos, a.npos) | a.fmask;
            if (u < a.n_units) v[r] = *reinterpret_cast<const float4*>(psi + base[r]);
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            const float2 y0 = cmul(diag_phase(a, base[r]), lo2(v[r]));
            const float2 y1 = cmul(diag_phase(a, base[r] | 1), hi2(v[r]));
            *reinterpret_cast<float4*>(psi + base[r]) = pack4(y0, y1);
        }
    } else {
        float2 v[U];
        uint64_t base[U];
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            base[r] = insert_zeros(u, a.pos, a.npos) | a.fmask;
            if (u < a.n_units) v[r] = psi[base[r]];
        }
#pragma unroll
        for (int r = 0; r < U; ++r) {
            const uint64_t u = u0 + (uint64_t)r * kBlock;
            if (u >= a.n_units) continue;
            psi[base[r]] = cmul(diag_phase(a, base[r]), v[r]);
        }
    }
}

// Every row := e_idx.
__global__ __launch_bounds__(kBlock) void k_basis(float2* p0, uint64_t N, uint64_t idx)
{
    float4* row = reinterpret_cast<float4*>(p0 + (uint64_t)blockIdx.y * N);
    const uint64_t n4 = N >> 1;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * kBlock) {
        float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i == (idx >> 1)) {
            if (idx & 1) z.z = 1.f;
            else z.x = 1.f;
        }
        row[i] = z;
    }
}

// Plain streaming copy (the bandwidth ceiling reference).
__global__ __launch_bounds__(kBlock) void k_copy(float4* __restrict__ dst, const float4* __restrict__ src, uint64_t n4)
{
    constexpr int U = 4;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock * U;
    for (uint64_t b = (uint64_t)blockIdx.x * kBlock * U + threadIdx.x; b < n4; b += stride) {
        float4 v[U];
#pragma unroll
        for (int r = 0; r < U; ++r)
            if (b + (uint64_t)r * kBlock < n4) v[r] = src[b + (uint64_t)r * kBlock];
#pragma unroll
        for (int r = 0; r < U; ++r)
            if (b + (uint64_t)r * kBlock < n4) dst[b + (uint64_t)r * kBlock] = v[r];
    }
}

void sort_small(int* v, int n)
{
    for (int i = 1; i < n; ++i)
        for (int j = i; j > 0 && v[j - 1] > v[j]; --j) std::swap(v[j - 1], v[j]);
}

constexpr int kUnroll = 2;

template <int K, int VEC>
void dispatch_gate(const KGate& a, int rows, hipStream_t st)
{
    const uint64_t per_block = (uint64_t)kBlock * kUnroll;
    const uint64_t blocks = (a.n_units + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_gate<K, VEC, kUnroll>), dim3((unsigned)blocks, rows), dim3(kBlock), 0, st, a);
    SV_HIP(hipGetLastError());
}

}  // namespace

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
    int lowest = 64;
    a.npos = 0;
    for (int j = 0; j < g.k; ++j) { a.pos[a.npos++] = g.targets[j]; lowest = std::min(lowest, g.targets[j]); }
    for (int j = 0; j < g.nc; ++j) {
        a.pos[a.npos++] = g.controls[j];
        a.cmask |= 1ull << g.controls[j];
        lowest = std::min(lowest, g.controls[j]);
    }
    sort_small(a.pos, a.npos);
    const uint64_t groups = 1ull << (n - g.k - g.nc);
    const int rows = g.rows.nrows;
    if (lowest >= 1 && groups >= 2) {
        a.n_units = groups >> 1;
        if (g.k == 1) dispatch_gate<1, 2>(a, rows, st);
        else dispatch_gate<2, 2>(a, rows, st);
    } else if (g.k == 1 && g.targets[0] == 0 && (g.nc == 0 || a.pos[1] >= 1)) {
        // pair (b, b|1) in one float4: the zero inserted at bit 0 is the target
        a.n_units = groups;
        dispatch_gate<1, 0>(a, rows, st);
    } else {
        a.n_units = groups;
        if (g.k == 1) dispatch_gate<1, 1>(a, rows, st);
        else dispatch_gate<2, 1>(a, rows, st);
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
    a.npos = d.nfixed;
    int lowest = 64;
    for (int j = 0; j < d.nfixed; ++j) {
        a.pos[j] = d.fixed[j];
        a.fmask |= 1ull << d.fixed[j];
        lowest = std::min(lowest, d.fixed[j]);
    }
    sort_small(a.pos, a.npos);
    a.nfree = d.nfree;
    for (int j = 0; j < d.nfree; ++j) a.fbit[j] = 1ull << d.freeq[j];
    for (int i = 0; i < (1 << d.nfree); ++i) a.ph[i] = d.ph[i];
    const uint64_t amps = 1ull << (n - d.nfixed);
    const uint64_t per_block = (uint64_t)kBlock * kUnroll;
    const int rows = d.rows.nrows;
    if (lowest >= 1 && amps >= 2) {
        a.n_units = amps >> 1;
        const uint64_t blocks = (a.n_units + per_block - 1) / per_block;
        hipLaunchKernelGGL((k_diag<2, kUnroll>), dim3((unsigned)blocks, rows), dim3(kBlock), 0, st, a);
    } else {
        a.n_units = amps;
        const uint64_t blocks = (a.n_units + per_block - 1) / per_block;
        hipLaunchKernelGGL((k_diag<1, kUnroll>), dim3((unsigned)blocks, rows), dim3(kBlock), 0, st, a);
    }
    SV_HIP(hipGetLastError());
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
    const uint64_t blocks = std::min<uint64_t>((n4 + kBlock * 4 - 1) / (kBlock * 4), 65536);
    hipLaunchKernelGGL(k_copy, dim3((unsigned)std::max<uint64_t>(blocks, 1)), dim3(kBlock), 0, st,
                       static_cast<float4*>(dst), static_cast<const float4*>(src), n4);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
