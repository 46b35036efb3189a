// k_adjoint.hip -- the adjoint backward: un-apply one gate from the state and
// from the co-state in the same sweep, and accumulate the gradient inner
// products of that gate's parameters in FP64.
//
// Sec. 4.4: for y = U x the backward recomputes the input as x = U^* y
// instead of storing it. With psi_l = U_l psi_{l-1}, lam_l = U_{l+1}^* ...
// U_L^* O psi_L, the derivative of L = <psi_L|O|psi_L> with respect to a
// parameter theta of U_l is 2 Re <lam_l| dU_l/dtheta |psi_{l-1}>
// = 2 Re <lam_l| G |psi_l> with G = dU_l/dtheta U_l^*. Every quantity is local
// to the gate's amplitude group, so one sweep reads psi_l and lam_l, adds
// Re <lam_l|G|psi_l> over the group, and writes psi_{l-1} = U^* psi_l and
// lam_{l-1} = U^* lam_l back.
#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

namespace {

struct KAdj {
    Rows psi;
    Rows lam;
    uint64_t n_units;
    uint64_t cmask;
    uint64_t moff[4];
    int npos;
    int pos[6];
    int nd;
    float2 uinv[16];
    double2 g[3][16];
};

__device__ __forceinline__ float2* mrow(const Rows& r, int row)
{
    return row < r.nrow0 ? r.p0 + (uint64_t)row * r.N : r.p1 + (uint64_t)(row - r.nrow0) * r.N;
}

template <int D>
__device__ __forceinline__ void adj_group(const KAdj& a, const float2 (&x)[D], const float2 (&l)[D],
                                          float2 (&xo)[D], float2 (&lo)[D], double (&acc)[3])
{
    // gradient terms: Re sum_i conj(l_i) (G_d x)_i in FP64
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d >= a.nd) break;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double mr = 0.0, mi = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const double2 g = a.g[d][i * D + j];
                mr += g.x * x[j].x - g.y * x[j].y;
                mi += g.x * x[j].y + g.y * x[j].x;
            }
            acc[d] += (double)l[i].x * mr + (double)l[i].y * mi;
        }
    }
    // un-apply
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float2 s = cmul(a.uinv[i * D], x[0]);
        float2 t = cmul(a.uinv[i * D], l[0]);
#pragma unroll
        for (int j = 1; j < D; ++j) {
            s = cfma(a.uinv[i * D + j], x[j], s);
            t = cfma(a.uinv[i * D + j], l[j], t);
        }
        xo[i] = s;
        lo[i] = t;
    }
}

// Forms (as for the plain sweeps): VEC2 = float4 members (no target/control
// on qubit 0), PAIR = one target at qubit 0 with the pair inside a float4,
// VEC1 = float2 members. Fixed grid with a grid-stride loop so each block's
// share (and the summation order) is fixed; two units per iteration for
// memory-level parallelism. NT = streaming accesses (whole lines written).
template <int K, int F, bool NT>
__global__ __launch_bounds__(kBlock) void k_adj(KAdj a, double* part)
{
    constexpr int D = 1 << K;
    constexpr int U = 2;
    const int row = blockIdx.y;
    float2* psi = mrow(a.psi, row);
    float2* lam = mrow(a.lam, row);
    double acc[3] = {0.0, 0.0, 0.0};
    const uint64_t stride = (uint64_t)gridDim.x * kBlock * U;
    const uint64_t blk = xcd_block(blockIdx.x, gridDim.x);
    for (uint64_t u0 = blk * kBlock * U + threadIdx.x; u0 < a.n_units; u0 += stride) {
        if constexpr (F == 2) {
            float4 vx[U][D], vl[U][D];
            uint64_t base[U];
#pragma unroll
            for (int r = 0; r < U; ++r) {
                const uint64_t u = u0 + (uint64_t)r * kBlock;
                base[r] = insert_zeros(u << 1, a.pos, a.npos) | a.cmask;
                if (u < a.n_units)
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        vx[r][j] = ld4<NT>(psi + (base[r] | a.moff[j]));
                        vl[r][j] = ld4<NT>(lam + (base[r] | a.moff[j]));
                    }
            }
#pragma unroll
            for (int r = 0; r < U; ++r) {
                if (u0 + (uint64_t)r * kBlock >= a.n_units) continue;
                float2 x0[D], l0[D], x1[D], l1[D], xo0[D], lo0[D], xo1[D], lo1[D];
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    x0[j] = lo2(vx[r][j]); x1[j] = hi2(vx[r][j]);
                    l0[j] = lo2(vl[r][j]); l1[j] = hi2(vl[r][j]);
                }
                adj_group<D>(a, x0, l0, xo0, lo0, acc);
                adj_group<D>(a, x1, l1, xo1, lo1, acc);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    st4<NT>(psi + (base[r] | a.moff[j]), pack4(xo0[j], xo1[j]));
                    st4<NT>(lam + (base[r] | a.moff[j]), pack4(lo0[j], lo1[j]));
                }
            }
        } else if constexpr (F == 0) {
            static_assert(K == 1, "pair form is for one target");
            float4 vx[U], vl[U];
            uint64_t base[U];
#pragma unroll
            for (int r = 0; r < U; ++r) {
                const uint64_t u = u0 + (uint64_t)r * kBlock;
                base[r] = insert_zeros(u, a.pos, a.npos) | a.cmask;
                if (u < a.n_units) {
                    vx[r] = ld4<NT>(psi + base[r]);
                    vl[r] = ld4<NT>(lam + base[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < U; ++r) {
                if (u0 + (uint64_t)r * kBlock >= a.n_units) continue;
                float2 x[2] = {lo2(vx[r]), hi2(vx[r])}, l[2] = {lo2(vl[r]), hi2(vl[r])}, xo[2], lo[2];
                adj_group<2>(a, x, l, xo, lo, acc);
                st4<NT>(psi + base[r], pack4(xo[0], xo[1]));
                st4<NT>(lam + base[r], pack4(lo[0], lo[1]));
            }
        } else {
            float2 x[U][D], l[U][D];
            uint64_t base[U];
#pragma unroll
            for (int r = 0; r < U; ++r) {
                const uint64_t u = u0 + (uint64_t)r * kBlock;
                base[r] = insert_zeros(u, a.pos, a.npos) | a.cmask;
                if (u < a.n_units)
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        x[r][j] = ld2<NT>(psi + (base[r] | a.moff[j]));
                        l[r][j] = ld2<NT>(lam + (base[r] | a.moff[j]));
                    }
            }
#pragma unroll
            for (int r = 0; r < U; ++r) {
                if (u0 + (uint64_t)r * kBlock >= a.n_units) continue;
                float2 xo[D], lo[D];
                adj_group<D>(a, x[r], l[r], xo, lo, acc);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    st2<NT>(psi + (base[r] | a.moff[j]), xo[j]);
                    st2<NT>(lam + (base[r] | a.moff[j]), lo[j]);
                }
            }
        }
    }
    block_sum<3>(acc);
    if (threadIdx.x == 0)
        for (int d = 0; d < a.nd; ++d) part[((uint64_t)row * a.nd + d) * gridDim.x + blockIdx.x] = acc[d];
}

// lam[c] = sum_t coeff_t i^{y_t} (-1)^{|(c ^ x_t) & z_t|} psi[c ^ x_t]
// (O psi for O = sum_t coeff_t P_t, written as a gather so every output
// amplitude is produced by one thread). Terms arrive sorted by x_mask: each
// distinct x_mask reads psi[c ^ x] once and applies the summed factor of its
// terms.
__global__ __launch_bounds__(kBlock) void k_pauli_sum(Rows rp, Rows rl, uint64_t N, const PauliTermDev* terms, int nt,
                                                   const double* coeff_rows, int zonly, int n)
{
    const int row = blockIdx.y;
    const double* crow = coeff_rows ? coeff_rows + (uint64_t)row * nt : nullptr;
    const float2* psi = mrow(rp, row);
    float2* lam = mrow(rl, row);
    if (zonly) {
        // every term is c Z_q: lambda_b = (G - 2 sum_{q: bit q of b} c_q) psi_b
        // with c_q summed per qubit (in term order) and per-byte tables of
        // the sums in LDS, so an amplitude takes one lookup per 8 qubits
        __shared__ double cq[64];
        __shared__ double tab[8][256];
        __shared__ double gsum;
        if (threadIdx.x == 0) {
            for (int q = 0; q < 64; ++q) cq[q] = 0.0;
            double g = 0.0;
            for (int t = 0; t < nt; ++t) {
                const PauliTermDev tm = terms[t];
                const double cf = crow ? crow[tm.orig] : tm.coeff;
                cq[__builtin_ctzll(tm.z_mask)] += cf;
                g += cf;
            }
            gsum = g;
        }
        __syncthreads();
        const int nb = (n + 7) / 8;
        for (int j = 0; j < nb; ++j) {
            double v = 0.0;
            for (int k = 0; k < 8; ++k)
                if ((threadIdx.x >> k) & 1) v += cq[8 * j + k];
            tab[j][threadIdx.x] = v;
        }
        __syncthreads();
        const double G = gsum;
        for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < N; c += (uint64_t)gridDim.x * kBlock) {
            double sb = 0.0;
            for (int j = 0; j < nb; ++j) sb += tab[j][(c >> (8 * j)) & 255];
            const double f = G - 2.0 * sb;
            const float2 v = psi[c];
            lam[c] = make_float2((float)(f * v.x), (float)(f * v.y));
        }
        return;
    }
    for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < N; c += (uint64_t)gridDim.x * kBlock) {
        double re = 0.0, im = 0.0;
        int t = 0;
        while (t < nt) {
            const uint64_t xm = ld_const(&terms[t].x_mask);
            const uint64_t src = c ^ xm;
            const float2 v = psi[src];
            double fr = 0.0, fi = 0.0;       // sum of coeff * sign * i^y over the terms of this x_mask
            for (; t < nt && ld_const(&terms[t].x_mask) == xm; ++t) {
                const PauliTermDev tm = ld_const(terms + t);     // uniform: the scalar cache
                const double cf = crow ? ld_const(crow + tm.orig) : tm.coeff;
                const double sg = (__popcll(src & tm.z_mask) & 1) ? -cf : cf;
                switch (tm.y_count & 3) {
                case 0: fr += sg; break;
                case 1: fi += sg; break;
                case 2: fr -= sg; break;
                default: fi -= sg; break;
                }
            }
            re += fr * v.x - fi * v.y;
            im += fr * v.y + fi * v.x;
        }
        lam[c] = make_float2((float)re, (float)im);
    }
}

}  // namespace

int adj_grid(int n, int k, int nc)
{
    const uint64_t units = 1ull << (n - k - nc);
    const uint64_t want = (units + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)device_info().cu_count * 8;
    return (int)std::max<uint64_t>(1, std::min(want, cap));
}

void launch_adj_step(const AdjLaunch& g, double* part, hipStream_t st)
{
    const int n = __builtin_ctzll(g.psi.N);
    KAdj a{};
    a.psi = g.psi;
    a.lam = g.lam;
    const int D = 1 << g.k;
    for (int i = 0; i < D * D; ++i) a.uinv[i] = g.uinv[i];
    a.nd = g.nd;
    for (int d = 0; d < g.nd; ++d)
        for (int i = 0; i < D * D; ++i) a.g[d][i] = g.g[d][i];
    for (int r = 0; r < D; ++r) {
        uint64_t off = 0;
        for (int j = 0; j < g.k; ++j)
            if ((r >> (g.k - 1 - j)) & 1) off |= 1ull << g.targets[j];
        a.moff[r] = off;
    }
    int lowest = 64;
    for (int j = 0; j < g.k; ++j) { a.pos[a.npos++] = g.targets[j]; lowest = std::min(lowest, g.targets[j]); }
    for (int j = 0; j < g.nc; ++j) {
        a.pos[a.npos++] = g.controls[j];
        a.cmask |= 1ull << g.controls[j];
        lowest = std::min(lowest, g.controls[j]);
    }
    for (int i = 1; i < a.npos; ++i)
        for (int j = i; j > 0 && a.pos[j - 1] > a.pos[j]; --j) std::swap(a.pos[j - 1], a.pos[j]);
    const uint64_t groups = 1ull << (n - g.k - g.nc);
    // every step of one backward uses the same grid: the partial-sum slots
    // are laid out with that stride
    const dim3 gd(g.grid, g.psi.nrows);
    const bool nt = a.pos[0] >= kFullLineQubit;
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, gd, dim3(kBlock), 0, st, a, part); };
    if (lowest >= 1 && groups >= 2) {
        a.n_units = groups >> 1;
        if (g.k == 1) nt ? go(k_adj<1, 2, true>) : go(k_adj<1, 2, false>);
        else nt ? go(k_adj<2, 2, true>) : go(k_adj<2, 2, false>);
    } else if (g.k == 1 && g.targets[0] == 0) {
        // pair (b, b|1) in one float4; lines are whole unless a control splits them
        a.n_units = groups;
        const bool nt_pair = a.npos < 2 || a.pos[1] >= kFullLineQubit;
        nt_pair ? go(k_adj<1, 0, true>) : go(k_adj<1, 0, false>);
    } else {
        a.n_units = groups;
        if (g.k == 1) go(k_adj<1, 1, false>);
        else go(k_adj<2, 1, false>);
    }
    SV_HIP(hipGetLastError());
}

// lambda = W psi for a diagonal observable W = diag(w) given per amplitude
// (w: [rows][N] doubles), the product taken in FP64 and rounded once.
__global__ __launch_bounds__(kBlock) void k_diag_lambda(Rows rp, Rows rl, uint64_t N, const double* __restrict__ w)
{
    const int row = blockIdx.y;
    const float2* psi = mrow(rp, row);
    float2* lam = mrow(rl, row);
    const double* wr = w + (uint64_t)row * N;
    for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < N; c += (uint64_t)gridDim.x * kBlock) {
        const float2 v = psi[c];
        const double f = wr[c];
        lam[c] = make_float2((float)(f * v.x), (float)(f * v.y));
    }
}

void launch_diag_lambda(const Rows& psi, const Rows& lam, int n, const double* w, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    const uint64_t blocks = std::min<uint64_t>((N + kBlock - 1) / kBlock, (uint64_t)device_info().cu_count * 16);
    hipLaunchKernelGGL(k_diag_lambda, dim3((unsigned)blocks, psi.nrows), dim3(kBlock), 0, st, psi, lam, N, w);
    SV_HIP(hipGetLastError());
}

void launch_apply_pauli_sum(const Rows& psi, const Rows& lam, int n, const PauliTermDev* terms, int nt,
                            const double* coeff_rows, hipStream_t st, bool zonly)
{
    const uint64_t N = 1ull << n;
    const uint64_t blocks = std::min<uint64_t>((N + kBlock - 1) / kBlock, (uint64_t)device_info().cu_count * 16);
    hipLaunchKernelGGL(k_pauli_sum, dim3((unsigned)blocks, psi.nrows), dim3(kBlock), 0, st, psi, lam, N, terms, nt,
                       coeff_rows, zonly ? 1 : 0, n);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
