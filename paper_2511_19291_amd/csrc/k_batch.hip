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

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ double2 d2(double re, double im) { return make_double2(re, im); }

// Gate matrix (first target = most significant index bit), complex128: the
// same definitions as the host gate math (rotations exp(-i t P / 2),
// OpenQASM U3, phase gate).
__device__ void dev_gate_matrix(int kind, const double* prm, double2* m)
{
    const double h = 0.70710678118654752440;
    const double2 z0 = d2(0, 0), o1 = d2(1, 0);
    for (int i = 0; i < kMatStride; ++i) m[i] = z0;
    auto set2 = [&](double2 a, double2 b, double2 c, double2 d) { m[0] = a; m[1] = b; m[2] = c; m[3] = d; };
    switch (kind) {
    case SV_H: set2(d2(h, 0), d2(h, 0), d2(h, 0), d2(-h, 0)); break;
    case SV_X: set2(z0, o1, o1, z0); break;
    case SV_Y: set2(z0, d2(0, -1), d2(0, 1), z0); break;
    case SV_Z: set2(o1, z0, z0, d2(-1, 0)); break;
    case SV_S: set2(o1, z0, z0, d2(0, 1)); break;
    case SV_SDG: set2(o1, z0, z0, d2(0, -1)); break;
    case SV_T: set2(o1, z0, z0, d2(h, h)); break;
    case SV_TDG: set2(o1, z0, z0, d2(h, -h)); break;
    case SV_SX: set2(d2(0.5, 0.5), d2(0.5, -0.5), d2(0.5, -0.5), d2(0.5, 0.5)); break;
    case SV_RX: case SV_RY: case SV_RZ: {
        double s, c;
        sincos(0.5 * prm[0], &s, &c);
        if (kind == SV_RX) set2(d2(c, 0), d2(0, -s), d2(0, -s), d2(c, 0));
        else if (kind == SV_RY) set2(d2(c, 0), d2(-s, 0), d2(s, 0), d2(c, 0));
        else set2(d2(c, -s), z0, z0, d2(c, s));
        break;
    }
    case SV_P: {
        double s, c;
        sincos(prm[0], &s, &c);
        set2(o1, z0, z0, d2(c, s));
        break;
    }
    case SV_U3: {
        double s, c, sf, cf, sl, cl, sfl, cfl;
        sincos(0.5 * prm[0], &s, &c);
        sincos(prm[1], &sf, &cf);
        sincos(prm[2], &sl, &cl);
        sincos(prm[1] + prm[2], &sfl, &cfl);
        set2(d2(c, 0), d2(-s * cl, -s * sl), d2(s * cf, s * sf), d2(c * cfl, c * sfl));
        break;
    }
    case SV_SWAP:
        m[0] = m[15] = o1;
        m[6] = m[9] = o1;
        break;
    case SV_RXX: case SV_RYY: case SV_RZZ: {
        double s, c;
        sincos(0.5 * prm[0], &s, &c);
        for (int i = 0; i < 4; ++i) m[i * 5] = d2(c, 0);
        if (kind == SV_RZZ) {
            // cos I - i sin Z(x)Z, Z(x)Z = diag(1, -1, -1, 1)
            m[0] = d2(c, -s); m[5] = d2(c, s); m[10] = d2(c, s); m[15] = d2(c, -s);
        } else if (kind == SV_RXX) {
            // X(x)X = antidiag(1, 1, 1, 1)
            m[3] = m[6] = m[9] = m[12] = d2(0, -s);
        } else {
            // Y(x)Y = antidiag(-1, 1, 1, -1)
            m[3] = d2(0, s); m[6] = d2(0, -s); m[9] = d2(0, -s); m[12] = d2(0, s);
        }
        break;
    }
    default: break;
    }
}

__device__ __forceinline__ void op_params(const BatchArgs& a, const BOp& op, double (&prm)[3])
{
    for (int q = 0; q < 3; ++q) prm[q] = op.p[q] >= 0 ? a.params[op.p[q]] : 0.0;
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b)
{
    return d2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int P>
__device__ __forceinline__ void dg1(double2 (&v)[16], const double2 (&m)[kMatStride], int cm)
{
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j & (1 << P)) continue;
        if ((j & cm) != cm) continue;
        const int j1 = j | (1 << P);
        const double2 x0 = v[j], x1 = v[j1];
        const double2 a0 = zmul(m[0], x0), b0 = zmul(m[1], x1), a1 = zmul(m[2], x0), b1 = zmul(m[3], x1);
        v[j] = d2(a0.x + b0.x, a0.y + b0.y);
        v[j1] = d2(a1.x + b1.x, a1.y + b1.y);
    }
}

template <int P0, int P1>
__device__ __forceinline__ void dg2(double2 (&v)[16], const double2 (&m)[kMatStride], int cm)
{
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j & ((1 << P0) | (1 << P1))) continue;
        if ((j & cm) != cm) continue;
        const int o[4] = {j, j | (1 << P1), j | (1 << P0), j | (1 << P0) | (1 << P1)};
        double2 x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = v[o[r]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double2 acc = d2(0, 0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double2 t = zmul(m[r * 4 + q], x[q]);
                acc.x += t.x;
                acc.y += t.y;
            }
            v[o[r]] = acc;
        }
    }
}

// One gate of a phase on a 16-amplitude vector in FP64 (the register-phase
// convention: targets rt[], controls rcmask, bit i <-> the phase's qubit g[i]).
__device__ void phase_gate_d(double2 (&v)[16], const BOp& op, const double2 (&m)[kMatStride])
{
    const int cm = op.rcmask;
    if (op.nt == 1) {
        switch (op.rt[0]) {
        case 0: dg1<0>(v, m, cm); break;
        case 1: dg1<1>(v, m, cm); break;
        case 2: dg1<2>(v, m, cm); break;
        default: dg1<3>(v, m, cm); break;
        }
        return;
    }
    switch (op.rt[0] * 4 + op.rt[1]) {
    case 1: dg2<0, 1>(v, m, cm); break;
    case 2: dg2<0, 2>(v, m, cm); break;
    case 3: dg2<0, 3>(v, m, cm); break;
    case 4: dg2<1, 0>(v, m, cm); break;
    case 6: dg2<1, 2>(v, m, cm); break;
    case 7: dg2<1, 3>(v, m, cm); break;
    case 8: dg2<2, 0>(v, m, cm); break;
    case 9: dg2<2, 1>(v, m, cm); break;
    case 11: dg2<2, 3>(v, m, cm); break;
    case 12: dg2<3, 0>(v, m, cm); break;
    case 13: dg2<3, 1>(v, m, cm); break;
    default: dg2<3, 2>(v, m, cm); break;
    }
}

// Column c of a fused phase's unitary: the phase's gates applied in FP64 to
// the basis vector e_c of its 16-amplitude space (bit i of the index <->
// the phase's qubit g[i]), then scattered into the matrix-core operand
// layout of the phase (see fused_phase below for the layout).
__device__ void build_fragment_column(const BatchArgs& a, int f, int c)
{
    const BPhase ph = a.phases[a.frag_phase[f]];
    double2 v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = d2(j == c ? 1.0 : 0.0, 0.0);
    for (int oi = ph.op_begin; oi < ph.op_end; ++oi) {
        const BOp op = a.ops[oi];
        double prm[3];
        op_params(a, op, prm);
        double2 m[kMatStride];
        dev_gate_matrix(op.kind, prm, m);
        phase_gate_d(v, op, m);
    }
    // v = U e_c.
    if (a.phase_mode == kPhaseFp32) {
        // three real 16 x 16 products (Gauss): Ur, Ui and Ur + Ui, rows in the
        // order of the FP32 16 x 16 x 4 output (row 4 iq + r <-> amplitude
        // 4 r + iq), as A operands: lane i + 16 (c & 3), step c >> 2
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int jo = 4 * (i & 3) + (i >> 2);
            const double ur = v[jo].x, ui = v[jo].y;
            float* fr = a.frag + ((size_t)f * 64 + i + 16 * (c & 3)) * kFragFloats;
            fr[0 * 4 + (c >> 2)] = (float)ur;
            fr[1 * 4 + (c >> 2)] = (float)ui;
            fr[2 * 4 + (c >> 2)] = (float)(ur + ui);
        }
        return;
    }
    // BF16 x3: real form [[Ur, -Ui], [Ui, Ur]]; row i (0..31) of the 32 x 32
    // operand is output component (i & 1) of amplitude jo(i) = 8 ((i >> 2) &
    // 1) + 2 (i >> 3) + ((i >> 1) & 1); the input column is (amplitude c,
    // component ci).
    const int lane_hi = 32 * (c >> 3);
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const int jo = 8 * ((i >> 2) & 1) + 2 * (i >> 3) + ((i >> 1) & 1);
        const double ur = v[jo].x, ui = v[jo].y;
        for (int ci = 0; ci < 2; ++ci) {
            const double e = (i & 1) == 0 ? (ci == 0 ? ur : -ui) : (ci == 0 ? ui : ur);
            float* fr = a.frag + ((size_t)f * 64 + lane_hi + i) * kFragFloats;
            const float ef = (float)e;
            const __bf16 hi = (__bf16)ef;
            const __bf16 lo = (__bf16)(ef - (float)hi);
            __bf16* fb = reinterpret_cast<__bf16*>(fr);
            fb[(ci * 2 + 0) * 8 + (c & 7)] = hi;
            fb[(ci * 2 + 1) * 8 + (c & 7)] = lo;
        }
    }
}

__global__ __launch_bounds__(256) void k_batch_prep(BatchArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < a.n_ops) {
        const BOp op = a.ops[i];
        double prm[3];
        op_params(a, op, prm);
        double2 m[kMatStride];
        dev_gate_matrix(op.kind, prm, m);
        for (int q = 0; q < kMatStride; ++q)
            a.mats[(size_t)i * kMatStride + q] = make_float2((float)m[q].x, (float)m[q].y);
    }
    if (i < a.n_frag * 16) build_fragment_column(a, i >> 4, i & 15);
    if (i < a.n_pass) a.done[i] = 0;
    if (i < a.n_circ) a.late[i] = 0;
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

// LDS layout of a tile: amplitude i sits at entry swz(i). An entry is 8
// bytes, so its bank pair is the entry index mod 16 (bits 0..3); XOR-ing tile
// bits 4..7 into bits 0..3 spreads the strided accesses of phases whose
// qubits include low tile bits over all bank pairs (sixteen lanes that take
// consecutive units then differ in bits 4..7 where they do not differ in bits
// 0..3). swz is linear over XOR, so swz(a | b) = swz(a) ^ swz(b) for disjoint
// bit sets, it is its own inverse, and it only permutes within aligned blocks
// of 16, so indices stay below 2^m. (XOR-ing bits 5..9 into bits 0..4 left
// bit 4 out of the bank pair: 1.9 conflict cycles per LDS instruction.)
__device__ __forceinline__ uint32_t swz(uint32_t i) { return i ^ ((i >> 4) & 15u); }

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
            const uint32_t w0 = swz(i0), w1 = swz(i1);
            const float2 x0 = s[w0], x1 = s[w1];
            s[w0] = cfma(m1, x1, cmul(m0, x0));
            s[w1] = cfma(m3, x1, cmul(m2, x0));
        }
    } else {
        float2 mm[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) mm[q] = mat[q];
        for (uint32_t g = threadIdx.x; g < groups; g += NT) {
            const uint32_t base = ins0(g, op.pos, op.np) | op.cmask;
            float2 x[4], y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = s[swz(base | op.off[r])];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float2 acc = cmul(mm[r * 4], x[0]);
#pragma unroll
                for (int c = 1; c < 4; ++c) acc = cfma(mm[r * 4 + c], x[c], acc);
                y[r] = acc;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) s[swz(base | op.off[r])] = y[r];
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

// Operand fragments of one fused phase for this lane: 64 bytes (FP32: 16
// floats; BF16 x3: the hi and lo parts of two 8-element operands).
struct Frag {
    float4 w[4];
};

// The fused-phase operands of one phase are 64 lanes x 64 bytes = 1024
// floats, identical for every wave: they are staged in LDS (two buffers, the
// next fused phase's copied in while the current one runs), and each lane
// reads its 64 bytes from there.
constexpr int kFragBlock = 64 * kFragFloats;

template <int NT>
struct FragCopy {
    static constexpr int W = kFragBlock / NT;    // floats per thread: 1, 2 or 4
    float v[W];
};

template <int NT>
__device__ __forceinline__ FragCopy<NT> frag_fetch(const BatchArgs& a, int f)
{
    FragCopy<NT> r;
    const float* p = a.frag + (size_t)f * kFragBlock + threadIdx.x * FragCopy<NT>::W;
#pragma unroll
    for (int q = 0; q < FragCopy<NT>::W; ++q) r.v[q] = p[q];
    return r;
}

template <int NT>
__device__ __forceinline__ void frag_put(float* buf, const FragCopy<NT>& r)
{
#pragma unroll
    for (int q = 0; q < FragCopy<NT>::W; ++q) buf[threadIdx.x * FragCopy<NT>::W + q] = r.v[q];
}

__device__ __forceinline__ Frag frag_lds(const float* buf, int lane)
{
    const float4* p = reinterpret_cast<const float4*>(buf + lane * kFragFloats);
    Frag r;
#pragma unroll
    for (int q = 0; q < 4; ++q) r.w[q] = p[q];
    return r;
}

__device__ __forceinline__ float frag_f(const Frag& fr, int s)
{
    const float4 v = fr.w[s >> 2];
    return (s & 3) == 0 ? v.x : (s & 3) == 1 ? v.y : (s & 3) == 2 ? v.z : v.w;
}

__device__ __forceinline__ bf16x8 frag_b(const Frag& fr, int idx)
{
    // idx = ci * 2 + (0 hi, 1 lo): 16 bytes
    const float4 v = fr.w[idx];
    return __builtin_bit_cast(bf16x8, v);
}

// The BF16 x3 products of one fused phase for two groups of 32 units
// (operand layouts as described for fused_phase).
template <int PM>
__device__ __forceinline__ void product2(const Frag& fr, const float2 (&xa)[8], const float2 (&xb)[8], f32x16& acca,
                                         f32x16& accb)
{
    {
#pragma unroll
        for (int ci = 0; ci < 2; ++ci) {
            bf16x8 ha, la, hb, lb;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float va = ci ? xa[q].y : xa[q].x, vb = ci ? xb[q].y : xb[q].x;
                ha[q] = (__bf16)va;
                la[q] = (__bf16)(va - (float)ha[q]);
                hb[q] = (__bf16)vb;
                lb[q] = (__bf16)(vb - (float)hb[q]);
            }
            const bf16x8 fh = frag_b(fr, ci * 2), fl = frag_b(fr, ci * 2 + 1);
            acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fl, ha, acca, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fl, hb, accb, 0, 0, 0);
            acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh, la, acca, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh, lb, accb, 0, 0, 0);
            acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh, ha, acca, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh, hb, accb, 0, 0, 0);
        }
    }
}

// A fused phase: every unit's 16 amplitudes y = U x with U the product of
// the phase's gates, on the matrix cores; a wave takes 32 units at a time.
//
// FP32 (Gauss's three real products): yr = Ur xr - Ui xi, yi = Ur xi + Ui xr
// from P1 = Ur xr, P2 = Ui xi, P3 = (Ur + Ui)(xr + xi) as yr = P1 - P2,
// yi = P3 - P1 - P2, each a 16 x 16 x 16 real product on
// v_mfma_f32_16x16x4_f32 (3/4 of the multiply-adds of the 32 x 32 real
// form). Per half-group of 16 units, lane (kq, u) (kq = lane / 16, unit u =
// lane % 16) supplies amplitude 4s + kq at step s and receives output row
// 4 kq + r, which the fragment builder maps to amplitude 4r + kq: each lane
// writes back exactly the four amplitudes it read.
//
// BF16 x3: the real product Y = M X with M = [[Ur, -Ui], [Ui, Ur]]
// (32 x 32) and X one 32-real column per unit (the 32 columns of one
// 32 x 32 x K product). Lane (h, u) (h = lane / 32, unit u = lane % 32 of
// the group) reads and writes amplitudes 8h .. 8h+7 of its unit: step s of
// v_mfma_f32_32x32x16_bf16 (K = 16) is component s of amplitudes 8h .. 8h+7,
// and output register r is component r & 1 of amplitude 8h + (r >> 1).
template <int NT, int PM>
__device__ __forceinline__ void fused_phase(float2* tile, int m, const BPhase& ph, const Frag& fr)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5;
    const uint32_t groups = 1u << (m - kRegBits - 5);
    const int g0 = ph.g[0], g1 = ph.g[1], g2 = ph.g[2], g3 = ph.g[3];
    if constexpr (PM == kPhaseFp32) {
        typedef float f32x4 __attribute__((ext_vector_type(4)));
        const int kq = lane >> 4, u16 = lane & 15;
        uint32_t offk[4];     // swizzled offsets of amplitudes 4s + kq
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int amp = 4 * st + kq;
            offk[st] = swz(((uint32_t)(amp & 1) << g0) | ((uint32_t)((amp >> 1) & 1) << g1) |
                           ((uint32_t)((amp >> 2) & 1) << g2) | ((uint32_t)((amp >> 3) & 1) << g3));
        }
        for (uint32_t grp = wave; grp < groups; grp += NW) {
            uint32_t ub[2];
            float2 x[2][4];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                uint32_t u = grp * 32 + nb * 16 + u16;
                u = ((u >> g0) << (g0 + 1)) | (u & ((1u << g0) - 1u));
                u = ((u >> g1) << (g1 + 1)) | (u & ((1u << g1) - 1u));
                u = ((u >> g2) << (g2 + 1)) | (u & ((1u << g2) - 1u));
                ub[nb] = swz(((u >> g3) << (g3 + 1)) | (u & ((1u << g3) - 1u)));
#pragma unroll
                for (int st = 0; st < 4; ++st) x[nb][st] = tile[ub[nb] ^ offk[st]];
            }
            f32x4 p1[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, p2[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}},
                  p3[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const float fr_r = frag_f(fr, st), fr_i = frag_f(fr, 4 + st), fr_s = frag_f(fr, 8 + st);
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
                    p1[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr_r, x[nb][st].x, p1[nb], 0, 0, 0);
                    p2[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr_i, x[nb][st].y, p2[nb], 0, 0, 0);
                    p3[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr_s, x[nb][st].x + x[nb][st].y, p3[nb], 0, 0, 0);
                }
            }
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    tile[ub[nb] ^ offk[r]] = make_float2(p1[nb][r] - p2[nb][r], p3[nb][r] - p1[nb][r] - p2[nb][r]);
        }
        return;
    }
    uint32_t offa[8];     // swizzled offsets of the lane's amplitudes within a unit
#pragma unroll
    for (int q = 0; q < 8; ++q)
        offa[q] = swz(((uint32_t)h << g3) | ((uint32_t)(q & 1) << g0) | ((uint32_t)((q >> 1) & 1) << g1) |
                      ((uint32_t)((q >> 2) & 1) << g2));
    // unit index -> (swizzled) tile index with zeros at the phase's qubits
    auto unit_base = [&](uint32_t grp) {
        uint32_t u = grp * 32 + (lane & 31);
        u = ((u >> g0) << (g0 + 1)) | (u & ((1u << g0) - 1u));
        u = ((u >> g1) << (g1 + 1)) | (u & ((1u << g1) - 1u));
        u = ((u >> g2) << (g2 + 1)) | (u & ((1u << g2) - 1u));
        return swz(((u >> g3) << (g3 + 1)) | (u & ((1u << g3) - 1u)));
    };
    // two groups per iteration (two independent accumulation chains)
    uint32_t grp = wave;
    for (; grp + NW < groups; grp += 2 * NW) {
        const uint32_t ua = unit_base(grp), ub = unit_base(grp + NW);
        float2 xa[8], xb[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) xa[q] = tile[ua ^ offa[q]];
#pragma unroll
        for (int q = 0; q < 8; ++q) xb[q] = tile[ub ^ offa[q]];
        f32x16 acca = {0}, accb = {0};
        product2<PM>(fr, xa, xb, acca, accb);
#pragma unroll
        for (int q = 0; q < 8; ++q) tile[ua ^ offa[q]] = make_float2(acca[2 * q], acca[2 * q + 1]);
#pragma unroll
        for (int q = 0; q < 8; ++q) tile[ub ^ offa[q]] = make_float2(accb[2 * q], accb[2 * q + 1]);
    }
    if (grp < groups) {
        const uint32_t ua = unit_base(grp);
        float2 xa[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) xa[q] = tile[ua ^ offa[q]];
        f32x16 acca = {0}, accb = {0};
        product2<PM>(fr, xa, xa, acca, accb);     // the second chain is discarded
#pragma unroll
        for (int q = 0; q < 8; ++q) tile[ua ^ offa[q]] = make_float2(acca[2 * q], acca[2 * q + 1]);
    }
}

// The scalar fields of a pass.
struct PassHead {
    int op_begin, op_end, phase_begin, phase_end, first_frag;
};

// One pass on the tile in LDS as register phases. A unit u < 2^(m-4) is the
// set of 16 amplitudes that share the complement bits u; the units of a phase
// are disjoint, so the threads take them in any order. The operands of the
// next fused phase are fetched while a fused phase runs (the pass's first
// ones while the tile is filled), so their latency overlaps that work.
template <int NT, int PM>
__device__ void run_phases(float2* tile, int m, const PassHead& ps, const BatchArgs& a, float* fragbuf)
{
    const uint32_t units = 1u << (m - kRegBits);
    int cur = 0;     // buffer holding the next fused phase's operands
    for (int hi = ps.phase_begin; hi < ps.phase_end; ++hi) {
        const BPhase ph = ld_const(a.phases + hi);
        if constexpr (PM != kPhaseGates) {
            if (ph.frag >= 0) {
                FragCopy<NT> nx{};
                if (ph.next_frag >= 0) nx = frag_fetch<NT>(a, ph.next_frag);
                const Frag fr = frag_lds(fragbuf + cur * kFragBlock, threadIdx.x & 63);
                fused_phase<NT, PM>(tile, m, ph, fr);
                if (ph.next_frag >= 0) frag_put<NT>(fragbuf + (cur ^ 1) * kFragBlock, nx);
                cur ^= 1;
                __syncthreads();
                continue;
            }
        }
        if (ph.g[0] < 0) {
            // a gate on more than four qubits: one LDS sweep
            for (int oi = ph.op_begin; oi < ph.op_end; ++oi) {
                lds_gate<NT>(tile, m, a.ops[oi], a.mats + (size_t)oi * kMatStride);
                __syncthreads();
            }
            continue;
        }
        uint32_t goff[kRegBits];      // swizzled offsets of the phase's qubits
#pragma unroll
        for (int i = 0; i < kRegBits; ++i) goff[i] = swz(1u << ph.g[i]);
        for (uint32_t u = threadIdx.x; u < units; u += NT) {
            // the unit index with zeros inserted at the phase's qubits (ascending)
            uint32_t base = u;
#pragma unroll
            for (int i = 0; i < kRegBits; ++i)
                base = ((base >> ph.g[i]) << (ph.g[i] + 1)) | (base & ((1u << ph.g[i]) - 1u));
            base = swz(base);
            float2 v[16];
            uint32_t off[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                uint32_t o = base;
#pragma unroll
                for (int i = 0; i < kRegBits; ++i)
                    if ((j >> i) & 1) o ^= goff[i];
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

// Sum of each of K per-thread values over the workgroup: red[w][i] holds
// wave w's sum of value i after the call.
template <int NT, int K>
__device__ __forceinline__ void wg_sum(double (&zs)[K], double (*red)[kZ])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int i = 0; i < K; ++i) zs[i] += __shfl_xor(zs[i], off, 64);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < K; ++i) red[wave][i] = zs[i];
    __syncthreads();
}

constexpr int log2i(int x) { return x <= 1 ? 0 : 1 + log2i(x / 2); }

// State offsets of a thread's tile elements (see the fill in k_batch);
// elements move in chunks of 2^CB.
template <int LB, int CB>
struct ElemOffsets {
    static constexpr int kHb = kMaxTileBits - 8;    // element bits: tile bits LB.. (LB >= 8)
    static constexpr int kChunk = 1 << CB;
    uint32_t off_t;                                  // this thread's own tile bits
    uint32_t hb[kHb];
    uint32_t hq[kChunk];                             // element bits 0..CB-1 of a chunk

    __device__ __forceinline__ ElemOffsets(const int* pos, int m)
    {
        const int hb_n = m > LB ? m - LB : 0;
        off_t = 0;
        for (int b = 0; b < m && b < LB; ++b)
            if ((threadIdx.x >> b) & 1) off_t |= 1u << pos[b];
#pragma unroll
        for (int i = 0; i < kHb; ++i) hb[i] = i < hb_n ? 1u << pos[LB + i] : 0u;
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            uint32_t o = 0;
#pragma unroll
            for (int i = 0; i < CB; ++i)
                if ((q >> i) & 1) o |= hb[i];
            hq[q] = o;
        }
    }
    // offset of chunk e0's element bits CB..
    __device__ __forceinline__ uint32_t chunk(int e0) const
    {
        uint32_t h0 = 0;
#pragma unroll
        for (int i = CB; i < kHb; ++i)
            if ((e0 >> i) & 1) h0 |= hb[i];
        return h0;
    }
};

template <int NT, int PM>
__global__ __launch_bounds__(NT) void k_batch(BatchArgs a)
{
    constexpr int LB = log2i(NT);
    constexpr int NW = NT / 64;
    constexpr int CB = NT >= 1024 ? 3 : 4;      // 2^CB elements per thread in flight (registers allow 16 below 1024)
    constexpr int kChunk = 1 << CB;
    using Offsets = ElemOffsets<LB, CB>;
    extern __shared__ float2 tile[];         // 2^m complex64, m <= the plan's tile width
    __shared__ double red[NW][kZ];
    __shared__ int s_pos[kMaxTileBits];      // the pass's tile qubits (LDS: indexed at run time)
    __shared__ int s_task, s_final, s_late;
    __shared__ __align__(16) float fragbuf[PM != kPhaseGates ? 2 * kFragBlock : 4];
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(a.counter, 1);
        __syncthreads();
        const int ti = __builtin_amdgcn_readfirstlane(s_task);   // uniform: table reads go through the scalar cache
        __syncthreads();
        if (ti >= a.n_tasks) break;
        const BTask tk = ld_const(a.tasks + ti);
        const BCirc c = ld_const(a.circ + tk.circ);
        const BPass& ps = a.pass[tk.pass];     // per-thread reads of pos[] below
        const PassHead hd = {ld_const(&ps.op_begin), ld_const(&ps.op_end), ld_const(&ps.phase_begin),
                             ld_const(&ps.phase_end), ld_const(&ps.first_frag)};
        const int m = c.m;
        if (threadIdx.x < kMaxTileBits) s_pos[threadIdx.x] = ps.pos[threadIdx.x];
        const uint32_t tsize = 1u << m;
        const bool first = tk.pass == c.pass_begin, last = tk.pass == c.pass_end - 1;
        if (threadIdx.x == 0) {
            s_late = 0;
            if (!first) {
                // every tile of the previous pass (handed out earlier) must be
                // done; a wait that gives up marks the circuit late, and the
                // circuit's output becomes NaN (its state is incomplete)
                const int limit = __hip_atomic_load(a.spin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                int late = limit < 0;
                for (int it = 0; !late && __hip_atomic_load(a.done + tk.pass - 1, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT) < c.ntiles;) {
                    __builtin_amdgcn_s_sleep(4);
                    if (++it > limit) late = 1;
                }
                if (late) {
                    s_late = 1;
                    __hip_atomic_fetch_or(a.late + tk.circ, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __threadfence();
            }
        }
        __syncthreads();
        const uint64_t base = insert_zeros((uint64_t)tk.tile, s_pos, m);
        // Element e of this thread is tile index l = threadIdx.x + (e << LB);
        // its state offset is base + off_t + hoff(e), hoff(e) = the OR of
        // 1 << pos[LB + i] over the set bits i of e. Elements move in chunks
        // of 2^CB so that a thread has that many memory accesses in flight. The offsets
        // are rebuilt from s_pos where they are used (fill, then store) so
        // that they hold no registers while the phases run.
        const int hb_n = m > LB ? m - LB : 0;
        const int per = 1 << hb_n;                  // elements per thread
        const bool active = threadIdx.x < tsize;    // m < LB: fewer amplitudes than threads
        // fill the tile (and stage the pass's first fused-phase operands)
        if constexpr (PM != kPhaseGates)
            if (hd.first_frag >= 0) frag_put<NT>(fragbuf, frag_fetch<NT>(a, hd.first_frag));
        if (active) {
            if (first) {
                for (int e = 0; e < per; ++e) {
                    const uint32_t l = threadIdx.x + ((uint32_t)e << LB);
                    tile[swz(l)] = make_float2(base == 0 && l == 0 ? 1.f : 0.f, 0.f);
                }
            } else {
                const Offsets eo(s_pos, m);
                const float2* st_t = a.arena + c.arena_off + base + eo.off_t;
                for (int e0 = 0; e0 < per; e0 += kChunk) {
                    const uint32_t h0 = eo.chunk(e0);
                    float2 v[kChunk];
#pragma unroll
                    for (int q = 0; q < kChunk; ++q)
                        if (q < per) v[q] = ld2<false>(st_t + (h0 | eo.hq[q]));
#pragma unroll
                    for (int q = 0; q < kChunk; ++q)
                        if (q < per) tile[swz(threadIdx.x + ((uint32_t)(e0 + q) << LB))] = v[q];
                }
            }
        }
        __syncthreads();
        if (hd.phase_end > hd.phase_begin) {
            run_phases<NT, PM>(tile, m, hd, a, fragbuf);
        } else {
            for (int oi = hd.op_begin; oi < hd.op_end; ++oi) {
                lds_gate<NT>(tile, m, a.ops[oi], a.mats + (size_t)oi * kMatStride);
                __syncthreads();
            }
        }
        if (last) {
            // probability sums per tile bit: S[b] = sum of p over the tile's
            // amplitudes with tile bit b set, S[kMaxTileBits] = sum of p. For
            // b < LB bit b is this thread's own, so only the element bits
            // (b >= LB) need per-amplitude work.
            constexpr int kS = kMaxTileBits + 1;
            constexpr int kHb = Offsets::kHb;
            double tot = 0.0, hs[kHb];
#pragma unroll
            for (int i = 0; i < kHb; ++i) hs[i] = 0.0;
            if (active)
                for (int e0 = 0; e0 < per; e0 += kChunk) {
#pragma unroll
                    for (int q = 0; q < kChunk; ++q) {
                        if (q >= per) continue;
                        const float2 v = tile[swz(threadIdx.x + ((uint32_t)(e0 + q) << LB))];
                        const double p = (double)v.x * v.x + (double)v.y * v.y;
                        tot += p;
#pragma unroll
                        for (int i = 0; i < kHb; ++i)
                            if (((e0 + q) >> i) & 1) hs[i] += p;
                    }
                }
            double zs[kS];
#pragma unroll
            for (int b = 0; b < kMaxTileBits; ++b) {
                if (b < LB) zs[b] = ((threadIdx.x >> b) & 1) ? tot : 0.0;
                else zs[b] = hs[b - LB];
            }
            zs[kMaxTileBits] = tot;
            wg_sum<NT, kS>(zs, red);
            // per qubit of the circuit: a tile qubit's sum, else the whole
            // tile's sum when the qubit's (fixed) bit in this tile is 1
            double zq = 0.0, tt = 0.0;
            const int i = threadIdx.x;
            if (i < kZ) {
                int bt = -1;
                for (int b = 0; b < m; ++b)
                    if (s_pos[b] == i) bt = b;
                for (int w = 0; w < NW; ++w) {
                    tt += red[w][kMaxTileBits];
                    if (bt >= 0) zq += red[w][bt];
                }
                if (i == kBatchMaxQubits) zq = tt;
                else if (bt < 0) zq = ((base >> i) & 1) ? tt : 0.0;
            }
            if (c.ntiles == 1) {
                if (i < SV_BATCH_OUT_STRIDE)
                    a.out[(size_t)c.out_idx * SV_BATCH_OUT_STRIDE + i] =
                        s_late ? __builtin_nan("") : (i < c.n ? tt - 2.0 * zq : 0.0);
            } else if (i < kZ) {
                a.zpart[(size_t)(c.zpart_off + tk.tile) * kZ + i] = s_late ? __builtin_nan("") : zq;
            }
        } else if (active) {
            const Offsets eo(s_pos, m);
            float2* st_t = a.arena + c.arena_off + base + eo.off_t;
            for (int e0 = 0; e0 < per; e0 += kChunk) {
                const uint32_t h0 = eo.chunk(e0);
                float2 v[kChunk];
#pragma unroll
                for (int q = 0; q < kChunk; ++q)
                    if (q < per) v[q] = tile[swz(threadIdx.x + ((uint32_t)(e0 + q) << LB))];
#pragma unroll
                for (int q = 0; q < kChunk; ++q)
                    if (q < per) st2<false>(st_t + (h0 | eo.hq[q]), v[q]);
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
            // every tile's partial is in: sum them in tile order. A tile of
            // any pass that gave up waiting flagged the circuit before it
            // counted itself done, so the flag is visible here.
            const int i = threadIdx.x;
            const bool late = __hip_atomic_load(a.late + tk.circ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            double t = 0.0, s = 0.0;
            if (i < c.n)
                for (int q = 0; q < c.ntiles; ++q) {
                    const double* zp = a.zpart + (size_t)(c.zpart_off + q) * kZ;
                    t += zp[kBatchMaxQubits];
                    s += zp[i];
                }
            a.out[(size_t)c.out_idx * SV_BATCH_OUT_STRIDE + i] =
                late ? __builtin_nan("") : (i < c.n ? t - 2.0 * s : 0.0);
        }
        __syncthreads();
    }
}

template <int NT>
void* batch_kernel(int phase_mode)
{
    switch (phase_mode) {
    case kPhaseFp32: return reinterpret_cast<void*>(&k_batch<NT, kPhaseFp32>);
    case kPhaseBf16x3: return reinterpret_cast<void*>(&k_batch<NT, kPhaseBf16x3>);
    default: return reinterpret_cast<void*>(&k_batch<NT, kPhaseGates>);
    }
}

void* batch_kernel_for(int threads, int phase_mode)
{
    return threads == 256 ? batch_kernel<256>(phase_mode)
           : threads == 512 ? batch_kernel<512>(phase_mode)
                            : batch_kernel<1024>(phase_mode);
}

}  // namespace

size_t batch_lds_bytes(int tile_bits)
{
    return (sizeof(float2) << tile_bits);
}

int batch_max_wg_per_cu(int threads, int tile_bits, int phase_mode)
{
    int nb = 0;
    const size_t lds = batch_lds_bytes(tile_bits);
    void* f = batch_kernel_for(threads, phase_mode);
    SV_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    SV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, threads, lds));
    return std::max(nb, 1);
}

void launch_batch(const BatchArgs& a, int grid, int threads, int tile_bits, hipStream_t st)
{
    const int items = std::max(std::max(std::max(a.n_ops, a.n_pass), std::max(a.n_frag * 16, 1)), a.n_circ);
    hipLaunchKernelGGL(k_batch_prep, dim3((items + 255) / 256), dim3(256), 0, st, a);
    SV_HIP(hipGetLastError());
    const size_t lds = batch_lds_bytes(tile_bits);
    void* f = batch_kernel_for(threads, a.phase_mode);
    void* args[] = {const_cast<BatchArgs*>(&a)};
    SV_HIP(hipLaunchKernel(f, dim3(grid), dim3(threads), args, lds, st));
}

}  // namespace sv
