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
//   4. each block that holds at least one shot is resolved by one wave:
//      every shot's chunk of 128 amplitudes (its mass known from step 1) is
//      read whole and coalesced, its probabilities scanned across the lanes
//      in a fixed order, and the shot's index found by a ballot (states
//      below 7 qubits: a lane per amplitude run, sequential walk).
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
// Blocks of at least 128 amplitudes (k_chunk_mass): one workgroup of eight
// waves per block (2^12 amplitudes: 32 chunks of 128), wave w reading chunks
// 4w .. 4w + 3 in memory order (one float4 per lane and chunk: lane l holds
// amplitudes 2l, 2l + 1), four loads in flight. The 64-lane sums of the four
// chunks are formed together by a reduce-scatter butterfly (xor 32, 16 halve
// the values a lane carries, xor 8, 4, 2, 1 finish one chunk per group of
// sixteen lanes): seven FP64 exchanges for four chunks, in a fixed order.
// The block's mass is the sum of its chunks' in chunk order. (Measured at 30
// qubits: eight chunks per wave and four waves per block 1.49 ms; one wave
// per block with two passes of sixteen chunks 1.85 ms.)
constexpr int kMassThreads = 512;
__global__ __launch_bounds__(kMassThreads) void k_chunk_mass(const float2* __restrict__ psi, int bb,
                                                            double* __restrict__ mass, double* __restrict__ csum)
{
    __shared__ double sh[1 << (kShotBits - kChunkBits)];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t nch = 1u << (bb - kChunkBits);
    const float4* p4 = reinterpret_cast<const float4*>(psi + ((uint64_t)blockIdx.x << bb));
    if ((uint32_t)(4 * w) < nch) {
        float4 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            v[i] = (uint32_t)(4 * w + i) < nch ? p4[(4 * w + i) * 64 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
        double t[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) t[i] = prob(make_float2(v[i].x, v[i].y)) + prob(make_float2(v[i].z, v[i].w));
        const bool b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1;
        double u2[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const double keep = b5 ? t[2 + j] : t[j], send = b5 ? t[j] : t[2 + j];
            u2[j] = keep + __shfl_xor(send, 32, 64);
        }
        double c = (b4 ? u2[1] : u2[0]) + __shfl_xor(b4 ? u2[0] : u2[1], 16, 64);
        c += __shfl_xor(c, 8, 64);
        c += __shfl_xor(c, 4, 64);
        c += __shfl_xor(c, 2, 64);
        c += __shfl_xor(c, 1, 64);
        const uint32_t ch = 4 * w + 2 * b5 + b4;            // the chunk this lane's group summed
        if ((lane & 15) == 0 && ch < nch) {
            sh[ch] = c;
            csum[((uint64_t)blockIdx.x << (kShotBits - kChunkBits)) + ch] = c;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (uint32_t c = 0; c < nch; ++c) m += sh[c];
        mass[blockIdx.x] = m;
    }
}

// Blocks below 128 amplitudes (states below 7 qubits): one workgroup sums a
// block.
__global__ __launch_bounds__(kST) void k_block_mass(const float2* __restrict__ psi, int bb, uint64_t nb,
                                                    double* __restrict__ mass, double* __restrict__ csum)
{
    __shared__ double sh[(1 << (kShotBits - kChunkBits)) > kST / 64 ? (1 << (kShotBits - kChunkBits)) : kST / 64];
    const uint64_t base = (uint64_t)blockIdx.x << bb;
    const uint32_t bs = 1u << bb;
    (void)nb;
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

// Blocks of at least 128 amplitudes: the shots, sorted by block, are taken
// eight at a time per wave, eight lanes per shot (lane i of a group). The
// group first finds the shot's chunk of 128 amplitudes from the block's chunk
// masses as k_block_mass stored them (lane i: chunks 4i .. 4i + 3, running
// sums in chunk order, then across the eight lanes in a fixed order): the
// first chunk whose running mass exceeds the shot's remainder. It then reads
// that chunk whole (lane i: amplitudes 16i .. 16i + 15, 128 contiguous bytes)
// and finds the first index of non-zero probability whose running sum (in
// index order) exceeds what remains. If rounding leaves none, the last index
// of non-zero probability in the chunk (past the last chunk: in the last
// chunk of non-zero mass). Only the chunks that hold a shot are read, and no
// index of zero probability is ever returned.
__device__ __forceinline__ double group_incl8(double v, int gi)
{
    // inclusive scan over the eight lanes of a group (Hillis-Steele, fixed order)
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
        const double t = __shfl_up(v, off, 8);
        if (gi >= off) v += t;
    }
    return v;
}

__device__ __forceinline__ void resolve_group(const float2* __restrict__ psi, int bb, const uint32_t* __restrict__ order,
                                              const uint32_t* __restrict__ blk, const double* __restrict__ rem,
                                              const double* __restrict__ csum, uint32_t j, bool valid, int lane,
                                              int64_t* __restrict__ out)
{
    const int gi = lane & 7;                          // lane within the shot's group
    const int gshift = lane & ~7;                     // first lane of the group
    const uint32_t nch = 1u << (bb - kChunkBits);
    const uint32_t sid = valid ? order[j] : 0u;
    const uint32_t b = valid ? blk[sid] : 0u;
    const double r = valid ? rem[sid] : 0.0;
    // chunk masses of the block: lane gi holds chunks 4 gi .. 4 gi + 3
    const double* cm = csum + ((uint64_t)b << (kShotBits - kChunkBits));
    double run[4], m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = (valid && (uint32_t)(4 * gi + k) < nch) ? cm[4 * gi + k] : 0.0;
    run[0] = m[0];
#pragma unroll
    for (int k = 1; k < 4; ++k) run[k] = run[k - 1] + m[k];
    const double lane_tot = run[3];
    // every cross-lane exchange below runs on all lanes (the groups diverge)
    const double incl = group_incl8(lane_tot, gi);
    const double up = __shfl_up(incl, 1, 8);
    const double pre = gi > 0 ? up : 0.0;
    int kc = -1;                                      // this lane's first chunk past r
#pragma unroll
    for (int k = 3; k >= 0; --k)
        if ((uint32_t)(4 * gi + k) < nch && pre + run[k] > r) kc = k;
    double mine_before = pre;                         // running mass before chunk 4 gi + kc
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (k < kc) mine_before = pre + run[k];
    int lastc = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (m[k] > 0.0) lastc = 4 * gi + k;
    const uint64_t gmask = 0xffull << gshift;
    const uint64_t found = __ballot(valid && kc >= 0) & gmask;
    const uint64_t nzc = __ballot(valid && lastc >= 0) & gmask;
    const int L = found ? __builtin_ctzll(found) - gshift : 0;
    const int H = nzc ? 63 - __builtin_clzll(nzc) - gshift : 0;
    const int kL = __shfl(kc, L, 8);
    const double excl = __shfl(mine_before, L, 8);
    const int lc = __shfl(lastc, H, 8);
    int chunk = found ? 4 * L + kL : lc;
    // rounding past the last chunk: the last chunk of non-zero mass, its last
    // non-zero index (need = 1e300 is never exceeded)
    const double need = found ? r - excl : 1e300;
    if (chunk < 0) chunk = 0;
    // the chunk, read 128 contiguous bytes per group and load: load t gives
    // lane gi amplitudes 16 t + 2 gi, 16 t + 2 gi + 1 (pair sum q[t]), so
    // sub-block t (amplitudes 16 t .. 16 t + 15) sits across the group
    const float4* c4 = reinterpret_cast<const float4*>(psi + ((uint64_t)b << bb) + ((uint64_t)chunk << kChunkBits)) + gi;
    float4 v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = valid ? c4[8 * t] : make_float4(0.f, 0.f, 0.f, 0.f);
    double p0[8], p1[8], q[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        p0[t] = prob(make_float2(v[t].x, v[t].y));
        p1[t] = prob(make_float2(v[t].z, v[t].w));
        q[t] = p0[t] + p1[t];
    }
    // sub-block totals by reduce-scatter over the group (lane gi ends with
    // sub-block gi's total), then their running sums across the group
    const bool g2 = (gi >> 2) & 1, g1 = (gi >> 1) & 1, g0 = gi & 1;
    double r4[4], r2[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double keep = g2 ? q[4 + j] : q[j], send = g2 ? q[j] : q[4 + j];
        r4[j] = keep + __shfl_xor(send, 4, 8);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const double keep = g1 ? r4[2 + j] : r4[j], send = g1 ? r4[j] : r4[2 + j];
        r2[j] = keep + __shfl_xor(send, 2, 8);
    }
    const double stot = (g0 ? r2[1] : r2[0]) + __shfl_xor(g0 ? r2[0] : r2[1], 1, 8);
    // (lane gi now holds sub-block gi's total)
    const double tot_in_order = stot;
    const double sincl = group_incl8(tot_in_order, gi);
    const double sup = __shfl_up(sincl, 1, 8);
    const double spre = gi > 0 ? sup : 0.0;
    // the sub-block holding the crossing: the first whose running sum exceeds need
    const uint64_t shit = __ballot(valid && sincl > need) & gmask;
    const uint64_t snz = __ballot(valid && tot_in_order > 0.0) & gmask;
    const int T = shit ? __builtin_ctzll(shit) - gshift : (snz ? 63 - __builtin_clzll(snz) - gshift : 0);
    const double sbefore = __shfl(spre, T, 8);
    const double need2 = shit ? need - sbefore : 1e300;
    // inside sub-block T: lane gi's pair (amplitudes 16 T + 2 gi, + 1)
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t)
        if (t == T) {
            a0 = p0[t];
            a1 = p1[t];
        }
    const double pincl = group_incl8(a0 + a1, gi);
    const double pup = __shfl_up(pincl, 1, 8);
    const double ppre = gi > 0 ? pup : 0.0;
    const bool c0 = a0 > 0.0 && ppre + a0 > need2;
    const bool c1 = a1 > 0.0 && ppre + a0 + a1 > need2;
    const uint64_t hit = __ballot(valid && (c0 || c1)) & gmask;
    const uint64_t anz = __ballot(valid && (a0 > 0.0 || a1 > 0.0)) & gmask;
    const uint64_t first0 = __ballot(valid && c0) & gmask;
    const uint64_t odd_nz = __ballot(valid && a1 > 0.0) & gmask;
    int idx = -1;
    if (hit) {
        const int L = __builtin_ctzll(hit);
        idx = 16 * T + 2 * (L - gshift) + (((first0 >> L) & 1) ? 0 : 1);
    } else if (anz) {
        const int H = 63 - __builtin_clzll(anz);
        idx = 16 * T + 2 * (H - gshift) + (((odd_nz >> H) & 1) ? 1 : 0);
    }
    if (valid && gi == 0)
        out[sid] = idx >= 0 ? (int64_t)(((uint64_t)b << bb) + ((uint64_t)chunk << kChunkBits) + (uint32_t)idx) : -1;
}

__global__ __launch_bounds__(kST) void k_shot_resolve_chunked(const float2* __restrict__ psi, int bb, uint32_t nb,
                                                              const uint32_t* __restrict__ cinc,
                                                              const uint32_t* __restrict__ order,
                                                              const uint32_t* __restrict__ blk,
                                                              const double* __restrict__ rem,
                                                              const double* __restrict__ csum,
                                                              int64_t* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const uint32_t total = cinc[nb - 1];              // shots that landed in a block
    const uint64_t nwaves = (uint64_t)gridDim.x * (kST / 64);
    for (uint64_t w = (uint64_t)blockIdx.x * (kST / 64) + (threadIdx.x >> 6); 8 * w < total; w += nwaves) {
        const uint64_t j = 8 * w + (lane >> 3);
        resolve_group(psi, bb, order, blk, rem, csum, (uint32_t)j, j < total, lane, out);
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
// ---------------------------------------------------------- <Z_i> from draws
//
// The shot estimate of every <Z_i> (Sec. 4.3, the measurement statistics of
// Sec. 2.2.1 sampled): E_i = 1 - 2 c_i / S with c_i the number of draws whose
// index has bit i set and S the number of draws with an index (the zero
// state's draws, -1, are left out). Counts are integers (wave ballots, one
// atomic add per wave and qubit), so the result is exact and independent of
// the order in which the waves finish.
__global__ __launch_bounds__(kST) void k_zero_u64(unsigned long long* __restrict__ x, int n)
{
    if ((int)threadIdx.x < n) x[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(kST) void k_shot_zcount(const int64_t* __restrict__ idx, int64_t shots, int n,
                                                     unsigned long long* __restrict__ cnt)
{
    const int lane = threadIdx.x & 63;
    unsigned long long mine = 0, valid = 0;        // lane q < n: draws with bit q set
    const int64_t stride = (int64_t)gridDim.x * kST;
    for (int64_t s0 = (int64_t)blockIdx.x * kST + (threadIdx.x & ~63); s0 < shots; s0 += stride) {
        const int64_t s = s0 + lane;
        const int64_t v = s < shots ? idx[s] : -1;
        const bool ok = v >= 0;
        valid += (unsigned long long)__popcll(__ballot(ok));
        for (int q = 0; q < n; ++q) {
            const unsigned long long b = __ballot(ok && ((v >> q) & 1));
            if (lane == q) mine += (unsigned long long)__popcll(b);
        }
    }
    if (lane < n && mine) atomicAdd(cnt + lane, mine);
    if (lane == 0 && valid) atomicAdd(cnt + n, valid);
}

__global__ void k_shot_zest(const unsigned long long* __restrict__ cnt, int n, double* __restrict__ est)
{
    const int q = threadIdx.x;
    if (q >= n) return;
    const unsigned long long s = cnt[n];
    est[q] = s ? 1.0 - 2.0 * ((double)cnt[q] / (double)s) : __builtin_nan("");
}

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

    if (bb >= kChunkBits)
        hipLaunchKernelGGL(k_chunk_mass, dim3((unsigned)nb), dim3(kMassThreads), 0, st, a.psi, bb, mass, csum);
    else
        hipLaunchKernelGGL(k_block_mass, dim3((unsigned)nb), dim3(kST), 0, st, a.psi, bb, (uint64_t)nb, mass, csum);
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
    if (bb >= kChunkBits) {
        const uint64_t groups = ((uint64_t)a.shots + 7) / 8;                // waves needed at most
        const unsigned cg = (unsigned)std::max<uint64_t>(
            1, std::min<uint64_t>((groups + 3) / 4, (uint64_t)device_info().cu_count * 16));
        hipLaunchKernelGGL(k_shot_resolve_chunked, dim3(cg), dim3(kST), 0, st, a.psi, bb, (uint32_t)nb, cinc, order,
                           blk, rem, csum, a.out);
    } else {
        hipLaunchKernelGGL(k_shot_resolve, dim3(rg), dim3(kST), 0, st, a.psi, bb, (uint32_t)nb, cinc, cnt, order,
                           rem, csum, a.out);
    }
    SV_HIP(hipGetLastError());
}

void launch_shot_zest(const int64_t* idx, int64_t shots, int n, void* scratch, double* est, hipStream_t st)
{
    unsigned long long* cnt = static_cast<unsigned long long*>(scratch);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(kST), 0, st, cnt, n + 1);
    SV_HIP(hipGetLastError());
    if (shots > 0) {
        const unsigned g = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>((shots + kST - 1) / kST, (int64_t)device_info().cu_count * 8));
        hipLaunchKernelGGL(k_shot_zcount, dim3(g), dim3(kST), 0, st, idx, shots, n, cnt);
        SV_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_shot_zest, dim3(1), dim3(64), 0, st, cnt, n, est);
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
