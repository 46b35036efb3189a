// k_shots.hip -- shot noise on the GPU state (Sec. 4.3).
//
// Exact sampling (Sec. 4.3.1). A shot is a draw of the basis index b with
// probability p_b = |psi_b|^2 / T; given the caller's uniform u it is the
// smallest b whose running probability sum exceeds u T (u T clamped below
// T). On the GPU:
//   1. block sums: the state is cut into blocks of 2^12 amplitudes and each
//      block's probability mass is summed in FP64 (one read sweep);
//   2. an inclusive scan of the block sums in a fixed order (so T and every
//      block's offset are deterministic);
//   3. each shot finds its block by binary search over the scanned sums
//      (an L2-resident array) and is bucketed by block (counting sort);
//   4. each block that holds at least one shot is read once more by one
//      wave: the lanes' masses are scanned with shuffles in a fixed order,
//      and each of its shots finds its lane by binary search and its index
//      by a sequential walk through that lane's amplitudes.
// The counts of the indices over all shots are one draw of the multinomial
// M(shots, p). This is the paper's hierarchical view restricted to one
// device: the blocks play the role of the groups whose masses q_j are known
// first, and the within-group draw is conditional on the group.
//
// Gaussian approximation (Sec. 4.3.2): y = shots p + sqrt(shots) D S z with
// D = diag(sqrt p), S = I - 2 v v^T the reflection that maps the last basis
// vector e to u = sqrt p (v = (e - u) / ||e - u||), z_last = 0. Applied
// matrix-free: S z = z - 2 v (v . z). One FP64 reduction sweep for T and
// sum_b |psi_b| z_b, then one elementwise sweep.
#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

namespace {

constexpr int kShotBits = 12;          // amplitudes per block
constexpr int kST = 256;               // threads per workgroup of the shot kernels
constexpr int kScanChunk = kST * 8;    // elements per workgroup of the scan

__device__ __forceinline__ double prob(float2 v) { return (double)v.x * v.x + (double)v.y * v.y; }

// Fixed-order sum over the workgroup (result valid in every thread).
__device__ double wg_sum256(double v, double* sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// Blocks of at least 2^kChunkBits amplitudes are also cut into chunks of
// 2^kChunkBits (128: one float4 per lane of a wave).
constexpr int kChunkBits = 7;
static_assert(kShotBits - kChunkBits <= 6, "a lane per chunk");

// 1. probability mass of each block of 2^bb amplitudes (bb <= kShotBits).
// With chunks: wave w's pass k reads chunk 4k + w in memory order (lane l:
// amplitudes 2l, 2l + 1 of the chunk); the chunk's mass is the wave's sum in
// a fixed order (butterfly; lane 0's value is stored), and the block's mass
// is the sum of its chunks' in chunk order.
__global__ __launch_bounds__(kST) void k_block_mass(const float2* __restrict__ psi, int bb, double* __restrict__ mass,
                                                    double* __restrict__ csum)
{
    __shared__ double sh[(1 << (kShotBits - kChunkBits)) > kST / 64 ? (1 << (kShotBits - kChunkBits)) : kST / 64];
    const uint64_t base = (uint64_t)blockIdx.x << bb;
    const uint32_t bs = 1u << bb;
    if (bb >= kChunkBits) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const uint32_t nch = 1u << (bb - kChunkBits);
        const float4* p4 = reinterpret_cast<const float4*>(psi + base);
        for (uint32_t c = w; c < nch; c += kST / 64) {
            const float4 v = p4[c * 64 + lane];
            double t = prob(make_float2(v.x, v.y)) + prob(make_float2(v.z, v.w));
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
            if (lane == 0) {
                sh[c] = t;
                csum[((uint64_t)blockIdx.x << (kShotBits - kChunkBits)) + c] = t;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = 0.0;
            for (uint32_t c = 0; c < nch; ++c) m += sh[c];
            mass[blockIdx.x] = m;
        }
        return;
    }
    double acc = 0.0;
    if (bs >= 2) {
        const float4* p4 = reinterpret_cast<const float4*>(psi + base);
        for (uint32_t i = threadIdx.x; i < bs / 2; i += kST) {
            const float4 v = p4[i];
            acc += prob(make_float2(v.x, v.y)) + prob(make_float2(v.z, v.w));
        }
    } else if (threadIdx.x == 0) {
        acc = prob(psi[base]);
    }
    const double s = wg_sum256(acc, sh);
    if (threadIdx.x == 0) mass[blockIdx.x] = s;
}

// 2. inclusive scan, chunks of kScanChunk elements: thread t owns the
// elements [8t, 8t + 8) of its chunk (sequential), then a Hillis-Steele scan
// of the 256 thread totals. Writes the chunk's total to tot[chunk].
template <class T>
__global__ __launch_bounds__(kST) void k_scan_chunk(T* __restrict__ x, uint64_t n, T* __restrict__ tot)
{
    __shared__ T sh[kST];
    const uint64_t c0 = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * 8;
    T v[8];
    T run = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        v[i] = c0 + i < n ? x[c0 + i] : (T)0;
        run += v[i];
        v[i] = run;
    }
    sh[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < kST; off <<= 1) {
        const T add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : (T)0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const T before = threadIdx.x > 0 ? sh[threadIdx.x - 1] : (T)0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (c0 + i < n) x[c0 + i] = before + v[i];
    if (threadIdx.x == kST - 1 && tot) tot[blockIdx.x] = sh[kST - 1];
}

template <class T>
__global__ __launch_bounds__(kST) void k_scan_add(T* __restrict__ x, uint64_t n, const T* __restrict__ tot)
{
    if (blockIdx.x == 0) return;
    const T off = tot[blockIdx.x - 1];
    const uint64_t c0 = (uint64_t)blockIdx.x * kScanChunk;
    for (uint32_t i = threadIdx.x; i < (uint32_t)kScanChunk; i += kST)
        if (c0 + i < n) x[c0 + i] += off;
}

__global__ __launch_bounds__(kST) void k_zero_u32(uint32_t* __restrict__ x, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kST + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kST) x[i] = 0;
}

// 3a. block of each shot: the first block whose inclusive mass exceeds t
__global__ __launch_bounds__(kST) void k_shot_locate(const double* __restrict__ pinc, uint32_t nb,
                                                     const double* __restrict__ u, int64_t shots,
                                                     uint32_t* __restrict__ blk, double* __restrict__ rem,
                                                     uint32_t* __restrict__ cnt, int64_t* __restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * kST + threadIdx.x;
    if (s >= shots) return;
    const double T = pinc[nb - 1];
    double t = u[s] * T;
    if (t >= T) t = nextafter(T, 0.0);
    uint32_t lo = 0, hi = nb;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (pinc[mid] > t) hi = mid;
        else lo = mid + 1;
    }
    if (lo == nb) {
        // zero state: no index has probability
        blk[s] = nb;
        out[s] = -1;
        return;
    }
    blk[s] = lo;
    rem[s] = t - (lo > 0 ? pinc[lo - 1] : 0.0);
    atomicAdd(cnt + lo, 1u);
}

// 3b. counting sort of the shots by block (order inside a bucket is free:
// each shot's result depends on its own uniform only)
__global__ __launch_bounds__(kST) void k_shot_scatter(const uint32_t* __restrict__ blk, int64_t shots, uint32_t nb,
                                                      const uint32_t* __restrict__ cinc, const uint32_t* __restrict__ cnt,
                                                      uint32_t* __restrict__ fill, uint32_t* __restrict__ order)
{
    const int64_t s = (int64_t)blockIdx.x * kST + threadIdx.x;
    if (s >= shots) return;
    const uint32_t b = blk[s];
    if (b >= nb) return;
    const uint32_t pos = cinc[b] - cnt[b] + atomicAdd(fill + b, 1u);
    order[pos] = (uint32_t)s;
}

// 4. per block with shots, one wave per block (blocks of at least 128
// amplitudes: resolve_chunked below). Smaller blocks (states below 7
// qubits): lane l owns the `per` contiguous amplitudes [per l, per (l + 1))
// of the block; the lanes' masses are scanned across the wave with
// shuffles in a fixed order. Each shot of the block finds its lane by binary
// search over the lanes' inclusive sums (shuffles: every lane takes part in
// every step), then its index by re-reading that lane's amplitudes in the
// same order: the first index whose running sum exceeds the remainder; if
// rounding leaves none, the last index of non-zero probability in the lane
// (or, past the last lane, in the block).
__device__ __forceinline__ double lane_prob(const float2* __restrict__ p, uint32_t i) { return prob(p[i]); }

// Last index of non-zero probability in chunk c of a block (-1 if none).
__device__ int chunk_last_nonzero(const float2* __restrict__ blk, uint32_t c)
{
    const float2* ch = blk + ((uint64_t)c << kChunkBits);
    int last = -1;
    for (int i = 0; i < (1 << kChunkBits); ++i)
        if (prob(ch[i]) > 0.0) last = (int)(c << kChunkBits) + i;
    return last;
}

// Blocks of at least 128 amplitudes: lane c takes chunk c's mass as
// k_block_mass stored it, and an inclusive scan over the lanes (fixed order)
// gives the chunks' running masses. Each shot (a lane per shot) finds its
// chunk by binary search over those sums and its index by reading that
// chunk in order (sixteen float4 loads in flight at a time): the first
// index whose running sum exceeds the remainder; if rounding leaves none,
// the last index of non-zero probability in the chunk (or, past the last
// chunk, in the block: in the last chunk of non-zero mass). Only the chunks
// that hold a shot are read.
__device__ __forceinline__ void resolve_chunked(const float2* __restrict__ blk, int bb, uint64_t base, int lane,
                                                const double* __restrict__ csum, uint32_t first, uint32_t nshot,
                                                const uint32_t* __restrict__ order, const double* __restrict__ rem,
                                                int64_t* __restrict__ out)
{
    const uint32_t nch = 1u << (bb - kChunkBits);
    const bool own = (uint32_t)lane < nch;
    const double mine = own ? csum[lane] : 0.0;
    const uint64_t nz = __ballot(own && mine > 0.0);        // chunks holding a non-zero probability
    double cincl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(cincl, off, 64);
        if (lane >= off) cincl += t;
    }
    for (uint32_t j0 = 0; j0 < nshot; j0 += 64) {
        const bool have = j0 + lane < nshot;
        const uint32_t s = have ? order[first + j0 + lane] : 0;
        const double r = have ? rem[s] : 0.0;
        // first chunk whose inclusive mass exceeds r
        uint32_t lo = 0, hi = nch;
#pragma unroll
        for (int step = 0; step < 7; ++step) {
            const uint32_t mid = lo + (hi - lo) / 2;
            const double im = __shfl(cincl, (int)min(mid, 63u), 64);
            if (lo < hi) {
                if (im > r) hi = mid;
                else lo = mid + 1;
            }
        }
        const double excl = __shfl(cincl, (int)(lo > 0 ? min(lo - 1, 63u) : 0u), 64);
        if (!have) continue;
        int idx = -1;
        if (lo < nch) {
            // the chunk in index order, 32 amplitudes (16 independent loads)
            // at a time
            const double need = r - (lo > 0 ? excl : 0.0);
            const float4* c4 = reinterpret_cast<const float4*>(blk + ((uint64_t)lo << kChunkBits));
            double acc = 0.0;
            int at = -1, lastnz = -1;
            for (uint32_t g = 0; g < (1u << kChunkBits) / 2 && at < 0; g += 16) {
                float4 w[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) w[q] = c4[g + q];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const double p0 = prob(make_float2(w[q].x, w[q].y)), p1 = prob(make_float2(w[q].z, w[q].w));
                    acc += p0;
                    if (p0 > 0.0) lastnz = (int)(2 * (g + q));
                    if (at < 0 && acc > need) at = (int)(2 * (g + q));
                    acc += p1;
                    if (p1 > 0.0) lastnz = (int)(2 * (g + q) + 1);
                    if (at < 0 && acc > need) at = (int)(2 * (g + q) + 1);
                }
            }
            // (when at < 0 the whole chunk was read, so lastnz is its last)
            const int pick = at >= 0 ? at : lastnz;
            if (pick >= 0) idx = (int)(lo << kChunkBits) + pick;
        }
        if (idx < 0 && nz) idx = chunk_last_nonzero(blk, 63u - (uint32_t)__builtin_clzll(nz));
        out[s] = idx >= 0 ? (int64_t)(base + (uint32_t)idx) : -1;
    }
}

__global__ __launch_bounds__(kST) void k_shot_resolve(const float2* __restrict__ psi, int bb, uint32_t nb,
                                                      const uint32_t* __restrict__ cinc, const uint32_t* __restrict__ cnt,
                                                      const uint32_t* __restrict__ order, const double* __restrict__ rem,
                                                      const double* __restrict__ csum, int64_t* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * (kST / 64) + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * (kST / 64);
    const uint32_t bs = 1u << bb;
    if (bb >= kChunkBits) {
        for (uint32_t b = wave; b < nb; b += nwaves) {
            const uint32_t nshot = cnt[b];
            if (nshot == 0) continue;
            const uint64_t co = (uint64_t)b << (kShotBits - kChunkBits);
            resolve_chunked(psi + ((uint64_t)b << bb), bb, (uint64_t)b << bb, lane, csum + co, cinc[b] - nshot,
                            nshot, order, rem, out);
        }
        return;
    }
    const uint32_t per = bs >= 64 ? bs / 64 : 1;
    const uint32_t nl = bs >= 64 ? 64 : bs;            // lanes that own amplitudes
    for (uint32_t b = wave; b < nb; b += nwaves) {
        const uint32_t nshot = cnt[b];
        if (nshot == 0) continue;
        const float2* blk = psi + ((uint64_t)b << bb);
        const float2* mine = blk + (uint64_t)lane * per;
        double sum = 0.0;
        int last = -1;
        if ((uint32_t)lane < nl) {
            if (per >= 2) {
                const float4* m4 = reinterpret_cast<const float4*>(mine);
                for (uint32_t i = 0; i < per / 2; ++i) {
                    const float4 v = m4[i];
                    const double p0 = prob(make_float2(v.x, v.y)), p1 = prob(make_float2(v.z, v.w));
                    sum += p0;
                    if (p0 > 0.0) last = (int)(lane * per + 2 * i);
                    sum += p1;
                    if (p1 > 0.0) last = (int)(lane * per + 2 * i + 1);
                }
            } else {
                sum = lane_prob(mine, 0);
                if (sum > 0.0) last = lane;
            }
        }
        // inclusive scan over the lanes (Hillis-Steele, fixed order)
        double incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        int blast = last;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) blast = max(blast, __shfl_xor(blast, off, 64));
        const uint32_t first = cinc[b] - nshot;
        for (uint32_t j0 = 0; j0 < nshot; j0 += 64) {
            const bool have = j0 + lane < nshot;
            const uint32_t s = have ? order[first + j0 + lane] : 0;
            const double r = have ? rem[s] : 0.0;
            // first lane whose inclusive sum exceeds r
            uint32_t lo = 0, hi = nl;
#pragma unroll
            for (int step = 0; step < 7; ++step) {
                const uint32_t mid = lo + (hi - lo) / 2;
                const double im = __shfl(incl, (int)min(mid, 63u), 64);
                if (lo < hi) {
                    if (im > r) hi = mid;
                    else lo = mid + 1;
                }
            }
            const double excl = __shfl(incl, (int)(lo > 0 ? min(lo - 1, 63u) : 0u), 64);
            if (!have) continue;
            int idx = blast;
            if (lo < nl) {
                const double need = r - (lo > 0 ? excl : 0.0);
                const float2* ch = blk + (uint64_t)lo * per;
                double run = 0.0;
                int lastc = -1;
                idx = -1;
                for (uint32_t i = 0; i < per; ++i) {
                    const double p = lane_prob(ch, i);
                    run += p;
                    if (p > 0.0) lastc = (int)(lo * per + i);
                    if (run > need) {
                        idx = (int)(lo * per + i);
                        break;
                    }
                }
                if (idx < 0) idx = lastc >= 0 ? lastc : blast;
            }
            out[s] = idx >= 0 ? (int64_t)(((uint64_t)b << bb) + (uint32_t)idx) : -1;
        }
    }
}

// Gaussian: partial sums of T = sum |psi|^2 and A = sum_{b < N-1} |psi_b| z_b
__global__ __launch_bounds__(kST) void k_gauss_partial(const float2* __restrict__ psi, const double* __restrict__ z,
                                                       uint64_t N, double* __restrict__ part)
{
    __shared__ double sh[kST / 64];
    double t = 0.0, a = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * kST + threadIdx.x; i < N / 2; i += (uint64_t)gridDim.x * kST) {
        const float4 v = reinterpret_cast<const float4*>(psi)[i];
        const double2 zz = reinterpret_cast<const double2*>(z)[i];
        const double p0 = prob(make_float2(v.x, v.y)), p1 = prob(make_float2(v.z, v.w));
        t += p0 + p1;
        a += sqrt(p0) * zz.x;
        if (2 * i + 1 < N - 1) a += sqrt(p1) * zz.y;
    }
    const double st = wg_sum256(t, sh);
    const double sa = wg_sum256(a, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = st;
        part[gridDim.x + blockIdx.x] = sa;
    }
}

// scalars: [0] T, [1] r = ||e - u||, [2] v . z
__global__ __launch_bounds__(kST) void k_gauss_final(const float2* __restrict__ psi, uint64_t N,
                                                     const double* __restrict__ part, int g, double* __restrict__ sc)
{
    __shared__ double sh[kST / 64];
    double t = 0.0, a = 0.0;
    for (int i = threadIdx.x; i < g; i += kST) {
        t += part[i];
        a += part[g + i];
    }
    const double T = wg_sum256(t, sh);
    const double A = wg_sum256(a, sh);
    if (threadIdx.x == 0) {
        const double pl = prob(psi[N - 1]);
        const double ul = sqrt(pl / T);
        // ||e - u||^2 = sum_{b < N-1} u_b^2 + (1 - u_last)^2
        const double r2 = (T - pl) / T + (1.0 - ul) * (1.0 - ul);
        const double r = sqrt(r2);
        sc[0] = T;
        sc[1] = r;
        // v . z = sum_{b < N-1} (-u_b / r) z_b (z_last = 0)
        sc[2] = r > 0.0 ? -(A / sqrt(T)) / r : 0.0;
    }
}

__global__ __launch_bounds__(kST) void k_gauss_y(const float2* __restrict__ psi, const double* __restrict__ z,
                                                 uint64_t N, double shots, const double* __restrict__ sc,
                                                 double* __restrict__ y)
{
    const uint64_t i = (uint64_t)blockIdx.x * kST + threadIdx.x;
    if (i >= N / 2) return;
    const double T = sc[0], r = sc[1], vz = sc[2];
    const double sq = sqrt(shots);
    const float4 v = reinterpret_cast<const float4*>(psi)[i];
    const double2 zz = reinterpret_cast<const double2*>(z)[i];
    double out[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint64_t b = 2 * i + h;
        const double p = prob(h ? make_float2(v.z, v.w) : make_float2(v.x, v.y)) / T;
        const double u = sqrt(p);
        const bool lastb = b == N - 1;
        const double vb = r > 0.0 ? ((lastb ? 1.0 : 0.0) - u) / r : 0.0;
        const double zb = lastb ? 0.0 : (h ? zz.y : zz.x);
        out[h] = shots * p + sq * u * (zb - 2.0 * vb * vz);
    }
    reinterpret_cast<double2*>(y)[i] = make_double2(out[0], out[1]);
}

// ---- Gaussian estimate of every <Z_i> and its backward (normals fixed).
// With p = q / T (q_b = |psi_b|^2), u = sqrt p, d = e - u, R = ||d||^2,
// K = d . z and y_b = shots p_b + sqrt(shots) u_b (z_b - 2 d_b K / R):
//   E_i = (1/shots) sum_b y_b s_i(b),   s_i(b) = 1 - 2 (bit i of b);
// for F = sum_i g_i E_i, c_b = sum_i g_i s_i(b), Q = sum_b c_b u_b d_b:
//   dF/dp_b = c_b + c_b K / (R sqrt shots)
//             + (c_b (S z)_b + 2 z_b Q / R - 4 d_b K Q / R^2) / (2 u_b sqrt shots)
//   (that last term 0 where u_b = 0), and
//   w_b = dF/dq_b = (dF/dp_b - sum_b' p_b' dF/dp_b') / T.
// y is the sampler's (same formula, same rounding); every sum is FP64 in a
// fixed order.

struct GzArgs {
    const float2* psi;
    const double* z;
    uint64_t N;
    int n;
    double shots;
    double g[SV_MAX_QUBITS];
    double G;                 // sum of g
    const double* sc;         // [0] T, [1] r = sqrt R, [2] v . z (v = d / r), [3] Q, [4] M
    double* part;
    double* w;
};

// y_b of the sampler
__device__ __forceinline__ double gz_y(double q, bool lastb, double zb, const double* sc, double shots, double sq)
{
    const double T = sc[0], r = sc[1], vz = sc[2];
    const double p = q / T;
    const double u = sqrt(p);
    const double vb = r > 0.0 ? ((lastb ? 1.0 : 0.0) - u) / r : 0.0;
    return shots * p + sq * u * (zb - 2.0 * vb * vz);
}

// c_b = G - 2 sum_{i: bit i of b} g_i from per-byte tables in LDS
__device__ __forceinline__ double gz_c(const double (*tab)[256], int nt, double G, uint64_t b)
{
    double s = 0.0;
    for (int j = 0; j < nt; ++j) s += tab[j][(b >> (8 * j)) & 255];
    return G - 2.0 * s;
}

__device__ void gz_tables(const GzArgs& a, double (*tab)[256], int nt)
{
    for (int j = 0; j < nt; ++j) {
        double s = 0.0;
        for (int k = 0; k < 8 && 8 * j + k < a.n; ++k)
            if ((threadIdx.x >> k) & 1) s += a.g[8 * j + k];
        tab[j][threadIdx.x] = s;
    }
    __syncthreads();
}

// E partials: per workgroup sum_b y_b and sum_{bit i of b} y_b for every i
__global__ __launch_bounds__(kST) void k_gz_est(GzArgs a)
{
    __shared__ double sh[kST / 64];
    const double sq = sqrt(a.shots);
    double tot = 0.0, acc[SV_MAX_QUBITS];
#pragma unroll
    for (int i = 0; i < SV_MAX_QUBITS; ++i) acc[i] = 0.0;
    for (uint64_t j = (uint64_t)blockIdx.x * kST + threadIdx.x; j < a.N / 2; j += (uint64_t)gridDim.x * kST) {
        const float4 v = reinterpret_cast<const float4*>(a.psi)[j];
        const double2 zz = reinterpret_cast<const double2*>(a.z)[j];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint64_t b = 2 * j + h;
            const bool lastb = b == a.N - 1;
            const double y = gz_y(prob(h ? make_float2(v.z, v.w) : make_float2(v.x, v.y)), lastb,
                                  lastb ? 0.0 : (h ? zz.y : zz.x), a.sc, a.shots, sq);
            tot += y;
#pragma unroll
            for (int i = 0; i < SV_MAX_QUBITS; ++i)
                if (i < a.n && ((b >> i) & 1)) acc[i] += y;
        }
    }
    const int stride = a.n + 1;
    const double st = wg_sum256(tot, sh);
    if (threadIdx.x == 0) a.part[(size_t)blockIdx.x * stride + a.n] = st;
#pragma unroll
    for (int i = 0; i < SV_MAX_QUBITS; ++i) {
        if (i < a.n) {     // uniform: every thread takes the same branches around the barriers
            const double si = wg_sum256(acc[i], sh);
            if (threadIdx.x == 0) a.part[(size_t)blockIdx.x * stride + i] = si;
        }
    }
}

// E_i = (tot - 2 acc_i) / shots from the partials, in workgroup order
__global__ __launch_bounds__(kST) void k_gz_est_final(const double* __restrict__ part, int g, int n, double shots,
                                                      double* __restrict__ est)
{
    __shared__ double sh[kST / 64];
    const int stride = n + 1;
    double tv = 0.0;
    for (int k = threadIdx.x; k < g; k += kST) tv += part[(size_t)k * stride + n];
    const double tot = wg_sum256(tv, sh);
    for (int i = 0; i < n; ++i) {
        double v = 0.0;
        for (int k = threadIdx.x; k < g; k += kST) v += part[(size_t)k * stride + i];
        const double si = wg_sum256(v, sh);
        if (threadIdx.x == 0) est[i] = (tot - 2.0 * si) / shots;
    }
}

// Q partials: sum_b c_b u_b d_b
__global__ __launch_bounds__(kST) void k_gz_q(GzArgs a)
{
    __shared__ double sh[kST / 64];
    __shared__ double tab[(SV_MAX_QUBITS + 7) / 8][256];
    const int nt = (a.n + 7) / 8;
    gz_tables(a, tab, nt);
    const double T = a.sc[0];
    double acc = 0.0;
    for (uint64_t b = (uint64_t)blockIdx.x * kST + threadIdx.x; b < a.N; b += (uint64_t)gridDim.x * kST) {
        const double u = sqrt(prob(a.psi[b]) / T);
        const double d = (b == a.N - 1 ? 1.0 : 0.0) - u;
        acc += gz_c(tab, nt, a.G, b) * u * d;
    }
    const double s = wg_sum256(acc, sh);
    if (threadIdx.x == 0) a.part[blockIdx.x] = s;
}

// w'_b = dF/dp_b (written to w) and partials of M = sum_b p_b w'_b
__global__ __launch_bounds__(kST) void k_gz_w(GzArgs a)
{
    __shared__ double sh[kST / 64];
    __shared__ double tab[(SV_MAX_QUBITS + 7) / 8][256];
    const int nt = (a.n + 7) / 8;
    gz_tables(a, tab, nt);
    const double T = a.sc[0], r = a.sc[1], Q = a.sc[3];
    const double R = r * r, K = r * a.sc[2];
    const double sq = sqrt(a.shots);
    double acc = 0.0;
    for (uint64_t b = (uint64_t)blockIdx.x * kST + threadIdx.x; b < a.N; b += (uint64_t)gridDim.x * kST) {
        const bool lastb = b == a.N - 1;
        const double p = prob(a.psi[b]) / T;
        const double u = sqrt(p);
        const double d = (lastb ? 1.0 : 0.0) - u;
        const double zb = lastb ? 0.0 : a.z[b];
        const double c = gz_c(tab, nt, a.G, b);
        double wp = c;
        if (R > 0.0) {
            const double sz = zb - 2.0 * d * K / R;
            wp += c * K / (R * sq);
            if (u > 0.0) wp += (c * sz + 2.0 * zb * Q / R - 4.0 * d * K * Q / (R * R)) / (2.0 * u * sq);
        } else if (u > 0.0) {
            wp += c * zb / (2.0 * u * sq);
        }
        a.w[b] = wp;
        acc += p * wp;
    }
    const double s = wg_sum256(acc, sh);
    if (threadIdx.x == 0) a.part[blockIdx.x] = s;
}

// a scalar from g partials, in workgroup order
__global__ __launch_bounds__(kST) void k_gz_scalar(const double* __restrict__ part, int g, double* __restrict__ out)
{
    __shared__ double sh[kST / 64];
    double v = 0.0;
    for (int k = threadIdx.x; k < g; k += kST) v += part[k];
    const double s = wg_sum256(v, sh);
    if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(kST) void k_gz_fix(double* __restrict__ w, uint64_t N, const double* __restrict__ sc)
{
    const double T = sc[0], M = sc[4];
    for (uint64_t b = (uint64_t)blockIdx.x * kST + threadIdx.x; b < N; b += (uint64_t)gridDim.x * kST)
        w[b] = (w[b] - M) / T;
}

template <class T>
void scan_inclusive(T* x, uint64_t n, T* tmp, hipStream_t st)
{
    const uint64_t chunks = (n + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_chunk<T>, dim3((unsigned)chunks), dim3(kST), 0, st, x, n, chunks > 1 ? tmp : (T*)nullptr);
    SV_HIP(hipGetLastError());
    if (chunks > 1) {
        scan_inclusive<T>(tmp, chunks, tmp + chunks, st);
        hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)chunks), dim3(kST), 0, st, x, n, (const T*)tmp);
        SV_HIP(hipGetLastError());
    }
}

// room for the recursive scan's chunk totals of an n-element scan
uint64_t scan_tmp(uint64_t n)
{
    uint64_t t = 0;
    while (n > (uint64_t)kScanChunk) {
        n = (n + kScanChunk - 1) / kScanChunk;
        t += n;
    }
    return t + 1;
}

int shot_block_bits(int n) { return n < kShotBits ? n : kShotBits; }

}  // namespace

size_t shot_scratch_bytes(int n, int64_t shots)
{
    const uint64_t nb = 1ull << (n - shot_block_bits(n));
    const uint64_t st = scan_tmp(nb);
    const uint64_t nch = (uint64_t)nb << (kShotBits - kChunkBits);   // chunk slots
    return (nb + st) * sizeof(double)                 // scanned masses + scan totals
           + (3 * nb + st) * sizeof(uint32_t)         // counts, fill, (count scan totals)
           + nch * sizeof(double)                     // chunk masses
           + (uint64_t)shots * (sizeof(double) + 2 * sizeof(uint32_t)) + 80;
}

void launch_sample_exact(const ShotLaunch& a, hipStream_t st)
{
    const int bb = shot_block_bits(a.n);
    const uint64_t nb = 1ull << (a.n - bb);
    const uint64_t stmp = scan_tmp(nb);
    char* p = static_cast<char*>(a.scratch);
    auto take = [&](size_t bytes) {
        char* q = p;
        p += (bytes + 7) & ~size_t(7);
        return q;
    };
    double* mass = reinterpret_cast<double*>(take(nb * sizeof(double)));
    double* dtmp = reinterpret_cast<double*>(take(stmp * sizeof(double)));
    uint32_t* cnt = reinterpret_cast<uint32_t*>(take(nb * sizeof(uint32_t)));
    uint32_t* cinc = reinterpret_cast<uint32_t*>(take(nb * sizeof(uint32_t)));
    uint32_t* fill = reinterpret_cast<uint32_t*>(take(nb * sizeof(uint32_t)));
    uint32_t* utmp = reinterpret_cast<uint32_t*>(take(stmp * sizeof(uint32_t)));
    double* rem = reinterpret_cast<double*>(take((size_t)a.shots * sizeof(double)));
    uint32_t* blk = reinterpret_cast<uint32_t*>(take((size_t)a.shots * sizeof(uint32_t)));
    uint32_t* order = reinterpret_cast<uint32_t*>(take((size_t)a.shots * sizeof(uint32_t)));
    const uint64_t nch = nb << (kShotBits - kChunkBits);
    double* csum = reinterpret_cast<double*>(take(nch * sizeof(double)));

    hipLaunchKernelGGL(k_block_mass, dim3((unsigned)nb), dim3(kST), 0, st, a.psi, bb, mass, csum);
    SV_HIP(hipGetLastError());
    scan_inclusive<double>(mass, nb, dtmp, st);
    if (a.shots == 0) return;
    const unsigned zg = (unsigned)std::min<uint64_t>((nb + kST - 1) / kST, 4096);
    hipLaunchKernelGGL(k_zero_u32, dim3(zg), dim3(kST), 0, st, cnt, nb);
    hipLaunchKernelGGL(k_zero_u32, dim3(zg), dim3(kST), 0, st, fill, nb);
    SV_HIP(hipGetLastError());
    const unsigned sg = (unsigned)((a.shots + kST - 1) / kST);
    hipLaunchKernelGGL(k_shot_locate, dim3(sg), dim3(kST), 0, st, mass, (uint32_t)nb, a.u, a.shots, blk, rem, cnt,
                       a.out);
    SV_HIP(hipGetLastError());
    SV_HIP(hipMemcpyAsync(cinc, cnt, nb * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    scan_inclusive<uint32_t>(cinc, nb, utmp, st);
    hipLaunchKernelGGL(k_shot_scatter, dim3(sg), dim3(kST), 0, st, blk, a.shots, (uint32_t)nb, cinc, cnt, fill, order);
    SV_HIP(hipGetLastError());
    const unsigned rg = (unsigned)std::min<uint64_t>((nb + 3) / 4, (uint64_t)device_info().cu_count * 8);
    hipLaunchKernelGGL(k_shot_resolve, dim3(rg), dim3(kST), 0, st, a.psi, bb, (uint32_t)nb, cinc, cnt, order, rem,
                       csum, a.out);
    SV_HIP(hipGetLastError());
}

uint64_t gauss_scratch_doubles(int n)
{
    (void)n;
    return 2 * (uint64_t)device_info().cu_count * 8 + 4;
}

void launch_sample_gaussian(const GaussLaunch& a, hipStream_t st)
{
    const uint64_t N = 1ull << a.n;
    const int g = (int)std::max<uint64_t>(1, std::min<uint64_t>((N / 2 + kST - 1) / kST, (uint64_t)device_info().cu_count * 8));
    double* part = a.scratch;
    double* sc = a.scratch + 2 * g;
    hipLaunchKernelGGL(k_gauss_partial, dim3(g), dim3(kST), 0, st, a.psi, a.z, N, part);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gauss_final, dim3(1), dim3(kST), 0, st, a.psi, N, part, g, sc);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gauss_y, dim3((unsigned)((N / 2 + kST - 1) / kST)), dim3(kST), 0, st, a.psi, a.z, N, a.shots,
                       sc, a.y);
    SV_HIP(hipGetLastError());
}

}  // namespace sv

namespace sv {

namespace {

int gz_grid(uint64_t N)
{
    return (int)std::max<uint64_t>(1, std::min<uint64_t>((N / 2 + kST - 1) / kST, (uint64_t)device_info().cu_count * 8));
}

// scratch: [0, 2g) T and A partials; [2g, 2g + 8) scalars; then the
// estimate partials (g (n + 1)) or the Q / M partials (g)
GzArgs gz_args(const GaussZLaunch& a, int g)
{
    GzArgs x{};
    x.psi = a.psi;
    x.z = a.z;
    x.N = 1ull << a.n;
    x.n = a.n;
    x.shots = a.shots;
    x.G = 0.0;
    for (int i = 0; i < a.n; ++i) {
        x.g[i] = a.g[i];
        x.G += a.g[i];
    }
    x.sc = a.scratch + 2 * g;
    x.part = a.scratch + 2 * g + 8;
    x.w = a.w;
    return x;
}

void gz_scalars(const GaussZLaunch& a, int g, hipStream_t st)
{
    const uint64_t N = 1ull << a.n;
    double* part = a.scratch;
    double* sc = a.scratch + 2 * g;
    hipLaunchKernelGGL(k_gauss_partial, dim3(g), dim3(kST), 0, st, a.psi, a.z, N, part);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gauss_final, dim3(1), dim3(kST), 0, st, a.psi, N, part, g, sc);
    SV_HIP(hipGetLastError());
}

}  // namespace

uint64_t gauss_z_scratch_doubles(int n)
{
    const uint64_t g = (uint64_t)device_info().cu_count * 8;
    return 2 * g + 8 + g * (uint64_t)(n + 1) + 8;
}

void launch_gauss_z(const GaussZLaunch& a, hipStream_t st)
{
    const int g = gz_grid(1ull << a.n);
    gz_scalars(a, g, st);
    const GzArgs x = gz_args(a, g);
    hipLaunchKernelGGL(k_gz_est, dim3(g), dim3(kST), 0, st, x);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gz_est_final, dim3(1), dim3(kST), 0, st, x.part, g, a.n, a.shots, a.est);
    SV_HIP(hipGetLastError());
}

void launch_gauss_z_backward(const GaussZLaunch& a, hipStream_t st)
{
    const uint64_t N = 1ull << a.n;
    const int g = gz_grid(N);
    gz_scalars(a, g, st);
    const GzArgs x = gz_args(a, g);
    double* sc = a.scratch + 2 * g;
    hipLaunchKernelGGL(k_gz_q, dim3(g), dim3(kST), 0, st, x);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gz_scalar, dim3(1), dim3(kST), 0, st, x.part, g, sc + 3);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gz_w, dim3(g), dim3(kST), 0, st, x);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gz_scalar, dim3(1), dim3(kST), 0, st, x.part, g, sc + 4);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gz_fix, dim3(g), dim3(kST), 0, st, a.w, N, x.sc);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
