// k_reduce.hip -- FP64 reductions over the state: Z expectations of every
// qubit in one sweep, general Pauli strings, inner products, drift.
//
// Measurement statistics follow Sec. 2.2.1: P(b) = |psi_b|^2 and
// <Z_i> = sum_b P(b) (1 - 2 b_i). Squares and sums are taken in FP64.
// Every reduction is two-stage with a fixed assignment of work to blocks and
// a fixed summation tree, so results are bitwise identical run to run.
#include "sv_device.h"
#include "sv_internal.h"

#include <map>
#include <mutex>

// Fixed partial-sum buffer of the allocation-free <Z_i> reduction: one copy
// per GPU, held until the process ends. Host code never passes this name to a
// kernel (on the host it is only a stand-in for the symbol); it passes the
// per-device address that static_zall_scratch() looks up.
static __device__ __align__(256) double scratch[sv::kStaticZallDoubles];

namespace sv {

namespace {

__device__ __forceinline__ const float2* crow(const Rows& r, int row)
{
    return row < r.nrow0 ? r.p0 + (uint64_t)row * r.N : r.p1 + (uint64_t)(row - r.nrow0) * r.N;
}

__device__ __forceinline__ double prob(float2 v)
{
    const double x = v.x, y = v.y;
    return fma(x, x, y * y);
}

// ---------------------------------------------------------- <Z_i> for all i
//
// Stage 1: block `blk` owns the tile of 2^tb consecutive amplitudes
// [blk 2^tb, (blk+1) 2^tb), 9 <= tb <= 14. Thread j reads float4 number
// f = j + 256 r (r < 2^(tb-9)), i.e. amplitudes l = 2 f + e. So inside the
// tile, bit 0 of l is e, bits 1..8 are the bits of j and bits 9.. are the
// bits of r. The block writes tot = sum P and S_i = sum_{bit i set} P for the
// tb tile bits. Bits above the tile are constant per block and are resolved
// in stage 2 from the block index.
__global__ __launch_bounds__(kBlock) void k_zall1(Rows rows, int tb, double* part, uint64_t nblk)
{
    const int row = blockIdx.y;
    const uint64_t blk = blockIdx.x;
    const float2* p = crow(rows, row) + (blk << tb);
    const int nr = 1 << (tb - 9);
    double tot = 0.0, s0 = 0.0, sr[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int r = 0; r < nr; ++r) {
        const float4 v = ld4(p + 2 * (threadIdx.x + kBlock * r));
        const double a = prob(lo2(v)), b = prob(hi2(v));
        const double ab = a + b;
        tot += ab;
        s0 += b;
#pragma unroll
        for (int k = 0; k < 5; ++k)
            if ((r >> k) & 1) sr[k] += ab;
    }
    double v[15];
    v[0] = tot;
    v[1] = s0;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[2 + k] = ((threadIdx.x >> k) & 1) ? tot : 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) v[10 + k] = sr[k];
    block_sum<15>(v);
    if (threadIdx.x == 0) {
        double* out = part + ((uint64_t)row * nblk + blk) * (tb + 1);
        for (int i = 0; i <= tb; ++i) out[i] = v[i];   // tot, S_0 .. S_{tb-1}
    }
}

// Small rows (n < 9): one block per row; S_i directly for every bit.
__global__ __launch_bounds__(kBlock) void k_zall1_small(Rows rows, int n, double* part)
{
    const int row = blockIdx.y;
    const float2* p = crow(rows, row);
    double v[9] = {0.0};
    for (uint64_t b = threadIdx.x; b < rows.N; b += kBlock) {
        const double pb = prob(p[b]);
        v[0] += pb;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (i < n && ((b >> i) & 1)) v[1 + i] += pb;
    }
    block_sum<9>(v);
    if (threadIdx.x == 0) {
        double* out = part + (uint64_t)row * (n + 1);
        for (int i = 0; i <= n; ++i) out[i] = v[i];
    }
}

// Stage 2: block (i, row) produces output i of one row. S_i for a tile bit
// is the sum of the blocks' S_i; for a bit above the tile it is the sum of the
// totals of the blocks whose index has bit i - tb. Every block also sums the
// totals (in the same fixed order), so out[row][i] = tot - 2 S_i and
// out[row][n] = tot come out of one pass.
__global__ __launch_bounds__(kBlock) void k_zall2(const double* part, int n, int tb, uint64_t nblk, double* out)
{
    const int i = blockIdx.x;
    const int row = blockIdx.y;
    const double* pr = part + (uint64_t)row * nblk * (tb + 1);
    double v[2] = {0.0, 0.0};   // tot, S_i
    for (uint64_t b = threadIdx.x; b < nblk; b += kBlock) {
        const double* q = pr + b * (tb + 1);
        v[0] += q[0];
        if (i < tb) v[1] += q[1 + i];
        else if (i < n && ((b >> (i - tb)) & 1)) v[1] += q[0];
    }
    block_sum<2>(v);
    if (threadIdx.x == 0) out[(uint64_t)row * (n + 1) + i] = i < n ? v[0] - 2.0 * v[1] : v[0];
}

// ---------------------------------------------------------- Pauli strings
//
// <P> = sum_b conj(psi[b ^ x]) i^{|x&z|} (-1)^{|b&z|} psi[b]. For x = 0 the
// summand is P(b) (-1)^{|b&z|}. For x != 0 the terms for b and b ^ x are
// complex conjugates of each other (P is Hermitian), so the sum runs over the
// bases b with bit h = 0 (h = highest bit of x) as 2 Re[...]. Terms sharing
// x are evaluated in one sweep.
struct KPauli {
    Rows rows;
    uint64_t x_mask;
    int hbit;
    int nt;
    uint64_t n_units;
    uint64_t z_mask[8];
    float2 ph[8];           // i^{|x & z_t|}: exact values in {1, i, -1, -i}
};

__device__ __forceinline__ double parity_sign(uint64_t v) { return (__popcll(v) & 1) ? -1.0 : 1.0; }

template <int NT>
__global__ __launch_bounds__(kBlock) void k_pauli1(KPauli a, double* part)
{
    const int row = blockIdx.y;
    const float2* p = crow(a.rows, row);
    double acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    if (a.x_mask == 0) {
        for (uint64_t b = (uint64_t)blockIdx.x * kBlock + threadIdx.x; b < a.n_units; b += stride) {
            const double pb = prob(p[b]);
#pragma unroll
            for (int t = 0; t < NT; ++t)
                if (t < a.nt) acc[t] += parity_sign(b & a.z_mask[t]) * pb;
        }
    } else {
        const int h = a.hbit;
        for (uint64_t u = (uint64_t)blockIdx.x * kBlock + threadIdx.x; u < a.n_units; u += stride) {
            const uint64_t b = ((u >> h) << (h + 1)) | (u & ((1ull << h) - 1ull));
            const float2 v = p[b], w = p[b ^ a.x_mask];
            // conj(w) * v in FP64
            const double re = (double)w.x * v.x + (double)w.y * v.y;
            const double im = (double)w.x * v.y - (double)w.y * v.x;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (t >= a.nt) continue;
                const double s = parity_sign(b & a.z_mask[t]);
                // Re[ph * s * (re + i im)]
                acc[t] += 2.0 * s * ((double)a.ph[t].x * re - (double)a.ph[t].y * im);
            }
        }
    }
    block_sum<NT>(acc);
    if (threadIdx.x == 0)
        for (int t = 0; t < a.nt; ++t) part[((uint64_t)row * a.nt + t) * gridDim.x + blockIdx.x] = acc[t];
}

// Sum `grid` partials per slot in a fixed order: out[s] = sum_b part[s*grid + b].
__global__ __launch_bounds__(kBlock) void k_sum_slots(const double* part, int grid, double* out)
{
    const int s = blockIdx.x;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < grid; b += kBlock) v[0] += part[(uint64_t)s * grid + b];
    block_sum<1>(v);
    if (threadIdx.x == 0) out[s] = v[0];
}

// ---------------------------------------------------------- inner product, drift

__global__ __launch_bounds__(kBlock) void k_inner1(Rows ra, Rows rb, uint64_t n4, double* part)
{
    const int row = blockIdx.y;
    const float4* pa = reinterpret_cast<const float4*>(crow(ra, row));
    const float4* pb = reinterpret_cast<const float4*>(crow(rb, row));
    double v[2] = {0.0, 0.0};
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * kBlock) {
        const float4 x = pa[i], y = pb[i];
        v[0] += (double)x.x * y.x + (double)x.y * y.y + (double)x.z * y.z + (double)x.w * y.w;
        v[1] += (double)x.x * y.y - (double)x.y * y.x + (double)x.z * y.w - (double)x.w * y.z;
    }
    block_sum<2>(v);
    if (threadIdx.x == 0) {
        part[((uint64_t)row * 2 + 0) * gridDim.x + blockIdx.x] = v[0];
        part[((uint64_t)row * 2 + 1) * gridDim.x + blockIdx.x] = v[1];
    }
}

__global__ __launch_bounds__(kBlock) void k_drift1(Rows ra, uint64_t n4, double* part)
{
    const int row = blockIdx.y;
    const float4* pa = reinterpret_cast<const float4*>(crow(ra, row));
    double v[1] = {0.0};
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * kBlock) {
        const float4 x = pa[i];
        const double re0 = (i == 0) ? (double)x.x - 1.0 : (double)x.x;
        v[0] += re0 * re0 + (double)x.y * x.y + (double)x.z * x.z + (double)x.w * x.w;
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) part[(uint64_t)row * gridDim.x + blockIdx.x] = v[0];
}

int sweep_grid(uint64_t units)
{
    const uint64_t want = (units + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)device_info().cu_count * 8;
    return (int)std::max<uint64_t>(1, std::min(want, cap));
}

int zall_tb(int n) { return n < 9 ? n : std::min(n, 14); }

}  // namespace

uint64_t zall_parts(int n, int rows)
{
    const int tb = zall_tb(n);
    return (uint64_t)rows * (1ull << (n - tb)) * (tb + 1);
}

void launch_zall(const Rows& r, int n, double* scratch, double* out, hipStream_t st)
{
    const int tb = zall_tb(n);
    const uint64_t nblk = 1ull << (n - tb);
    if (n < 9) {
        hipLaunchKernelGGL(k_zall1_small, dim3(1, r.nrows), dim3(kBlock), 0, st, r, n, scratch);
    } else {
        hipLaunchKernelGGL(k_zall1, dim3((unsigned)nblk, r.nrows), dim3(kBlock), 0, st, r, tb, scratch, nblk);
    }
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_zall2, dim3(n + 1, r.nrows), dim3(kBlock), 0, st, scratch, n, tb, nblk, out);
    SV_HIP(hipGetLastError());
}

uint64_t pauli_parts(int n, int rows, int nt)
{
    return (uint64_t)rows * nt * sweep_grid(1ull << n);
}

void launch_pauli_group(const Rows& r, int n, const PauliGroup& g, double* scratch, double* out, hipStream_t st)
{
    KPauli a{};
    a.rows = r;
    a.x_mask = g.x_mask;
    a.nt = g.nt;
    a.hbit = g.x_mask ? 63 - __builtin_clzll(g.x_mask) : -1;
    a.n_units = g.x_mask ? (1ull << (n - 1)) : (1ull << n);
    static const float2 iy[4] = {{1.f, 0.f}, {0.f, 1.f}, {-1.f, 0.f}, {0.f, -1.f}};
    for (int t = 0; t < g.nt; ++t) {
        a.z_mask[t] = g.z_mask[t];
        a.ph[t] = iy[g.y_count[t] & 3];
    }
    const int grid = sweep_grid(a.n_units);
    if (g.nt <= 1)
        hipLaunchKernelGGL(k_pauli1<1>, dim3(grid, r.nrows), dim3(kBlock), 0, st, a, scratch);
    else if (g.nt <= 4)
        hipLaunchKernelGGL(k_pauli1<4>, dim3(grid, r.nrows), dim3(kBlock), 0, st, a, scratch);
    else
        hipLaunchKernelGGL(k_pauli1<8>, dim3(grid, r.nrows), dim3(kBlock), 0, st, a, scratch);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_slots, dim3(r.nrows * g.nt), dim3(kBlock), 0, st, scratch, grid, out);
    SV_HIP(hipGetLastError());
}

uint64_t inner_parts(int n, int rows) { return (uint64_t)rows * 2 * sweep_grid(1ull << (n - 1)); }

void launch_inner(const Rows& a, const Rows& b, int n, double* scratch, double* out, hipStream_t st)
{
    const uint64_t n4 = 1ull << (n - 1);
    const int grid = sweep_grid(n4);
    hipLaunchKernelGGL(k_inner1, dim3(grid, a.nrows), dim3(kBlock), 0, st, a, b, n4, scratch);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_slots, dim3(a.nrows * 2), dim3(kBlock), 0, st, scratch, grid, out);
    SV_HIP(hipGetLastError());
}

uint64_t drift_parts(int n, int rows) { return (uint64_t)rows * sweep_grid(1ull << (n - 1)); }

void launch_drift(const Rows& a, int n, double* scratch, double* out, hipStream_t st)
{
    const uint64_t n4 = 1ull << (n - 1);
    const int grid = sweep_grid(n4);
    hipLaunchKernelGGL(k_drift1, dim3(grid, a.nrows), dim3(kBlock), 0, st, a, n4, scratch);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_slots, dim3(a.nrows), dim3(kBlock), 0, st, scratch, grid, out);
    SV_HIP(hipGetLastError());
}

void launch_sum_slots(const double* part, int grid, int nslots, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_slots, dim3(nslots), dim3(kBlock), 0, st, part, grid, out);
    SV_HIP(hipGetLastError());
}

double* static_zall_scratch()
{
    static std::mutex mu;
    static std::map<int, double*> addr;   // device -> address of its copy of `scratch`
    int dev = 0;
    SV_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* p = nullptr;
    SV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) fail(SV_ERR_HIP, "hipGetSymbolAddress returned a null address for the Z scratch");
    addr.emplace(dev, static_cast<double*>(p));
    return static_cast<double*>(p);
}

}  // namespace sv
