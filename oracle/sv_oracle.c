/*
 * sv_oracle.c -- plain complex128 CPU reference of the state-vector method.
 *
 * TEST INFRASTRUCTURE. This is the oracle that the GPU library is checked
 * against. Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the GPU library never does, and the two share no code.
 *
 * Everything here is the plain definition, written for a reader to check
 * by eye against the paper:
 *   - state: psi in C^(2^n), one complex128 per basis index b; qubit q is
 *     bit q of b (qubit 0 = least significant). (Sec. 2.2.1, Sec. 4.1.1)
 *   - gate (M, Q): M is 2^k x 2^k, Q the ordered target list. MoveDim moves
 *     the dimensions Q to the front in order, so Q[0] is the most significant
 *     bit of M's row/column index; the product mm(M, X) then runs over the
 *     remaining indices. (Sec. 4.1.1, Alg. 1 and Alg. 2 give the same result)
 *     Controls C: the gate acts only where every control bit is 1.
 *   - Z-basis probabilities |psi_b|^2 and expectation values. (Sec. 2.2.1)
 * Reductions are Neumaier-compensated double sums over a fixed chunking, so
 * results do not depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double complex cplx;

#define ORC_MAX_K 6

/* ---------------------------------------------------------------- gates */

/* Pauli generator P of a rotation kind (rx ry rz: X Y Z on one qubit;
 * rxx ryy rzz: X(x)X, Y(x)Y, Z(x)Z on two). Returns k, or -1 otherwise. */
static int rot_generator(const char* kind, cplx* p)
{
    cplx p1[4];
    int k;
    if (!strcmp(kind, "rx") || !strcmp(kind, "rxx")) { p1[0] = 0; p1[1] = 1; p1[2] = 1; p1[3] = 0; }
    else if (!strcmp(kind, "ry") || !strcmp(kind, "ryy")) { p1[0] = 0; p1[1] = -I; p1[2] = I; p1[3] = 0; }
    else if (!strcmp(kind, "rz") || !strcmp(kind, "rzz")) { p1[0] = 1; p1[1] = 0; p1[2] = 0; p1[3] = -1; }
    else return -1;
    k = (int)strlen(kind) - 1;                       /* "rx" -> 1, "rxx" -> 2 */
    if (k == 1) {
        for (int i = 0; i < 4; ++i) p[i] = p1[i];
    } else {
        /* Kronecker product: row r = (r1 r0), column q = (q1 q0), with the
         * first target as the most significant bit. */
        for (int r = 0; r < 4; ++r)
            for (int q = 0; q < 4; ++q)
                p[r * 4 + q] = p1[(r >> 1) * 2 + (q >> 1)] * p1[(r & 1) * 2 + (q & 1)];
    }
    return k;
}

/* Matrix of a named gate kind, row-major, Q[0] = most significant bit of
 * the index. Returns k (number of targets), or -1 for an unknown kind.
 * Rotations are R_P(theta) = exp(-i theta P / 2) = cos(theta/2) I
 * - i sin(theta/2) P since P^2 = I (the Pauli rotations of Sec. 3); u3 is
 * the OpenQASM 2 form; p(l) = diag(1, e^{il}). */
int orc_gate_matrix(const char* kind, const double* prm, cplx* m)
{
    const double r2 = 1.0 / sqrt(2.0);
    cplx p[16];
    int k = rot_generator(kind, p);
    if (k > 0) {
        int d = 1 << k;
        double c = cos(prm[0] / 2), s = sin(prm[0] / 2);
        for (int r = 0; r < d; ++r)
            for (int q = 0; q < d; ++q)
                m[r * d + q] = (r == q ? c : 0.0) - I * s * p[r * d + q];
        return k;
    }
    if (!strcmp(kind, "h"))   { m[0] = r2; m[1] = r2; m[2] = r2; m[3] = -r2; return 1; }
    if (!strcmp(kind, "x"))   { m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; return 1; }
    if (!strcmp(kind, "y"))   { m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; return 1; }
    if (!strcmp(kind, "z"))   { m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1; return 1; }
    if (!strcmp(kind, "s"))   { m[0] = 1; m[1] = 0; m[2] = 0; m[3] = I; return 1; }
    if (!strcmp(kind, "sdg")) { m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -I; return 1; }
    if (!strcmp(kind, "t"))   { m[0] = 1; m[1] = 0; m[2] = 0; m[3] = (1 + I) * r2; return 1; }
    if (!strcmp(kind, "tdg")) { m[0] = 1; m[1] = 0; m[2] = 0; m[3] = (1 - I) * r2; return 1; }
    if (!strcmp(kind, "sx"))  {
        m[0] = 0.5 * (1 + I); m[1] = 0.5 * (1 - I);
        m[2] = 0.5 * (1 - I); m[3] = 0.5 * (1 + I); return 1;
    }
    if (!strcmp(kind, "p")) { m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(I * prm[0]); return 1; }
    if (!strcmp(kind, "u3")) {
        double c = cos(prm[0] / 2), s = sin(prm[0] / 2), f = prm[1], l = prm[2];
        m[0] = c; m[1] = -cexp(I * l) * s; m[2] = cexp(I * f) * s; m[3] = cexp(I * (f + l)) * c;
        return 1;
    }
    if (!strcmp(kind, "swap")) {
        for (int i = 0; i < 16; ++i) m[i] = 0;
        m[0 * 4 + 0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[3 * 4 + 3] = 1;
        return 2;
    }
    return -1;
}

/* d M / d prm[j] for the parameterised kinds, same layout as the matrix.
 * Returns k, or -1 if the kind has no parameter j. */
int orc_gate_dmatrix(const char* kind, const double* prm, int j, cplx* m)
{
    cplx p[16];
    int k = rot_generator(kind, p);
    if (k > 0) {
        if (j != 0) return -1;
        /* d/dtheta [cos(theta/2) I - i sin(theta/2) P] */
        int d = 1 << k;
        double dc = -0.5 * sin(prm[0] / 2), ds = 0.5 * cos(prm[0] / 2);
        for (int r = 0; r < d; ++r)
            for (int q = 0; q < d; ++q)
                m[r * d + q] = (r == q ? dc : 0.0) - I * ds * p[r * d + q];
        return k;
    }
    if (!strcmp(kind, "p")) {
        if (j != 0) return -1;
        m[0] = 0; m[1] = 0; m[2] = 0; m[3] = I * cexp(I * prm[0]);
        return 1;
    }
    if (!strcmp(kind, "u3")) {
        double c = cos(prm[0] / 2), s = sin(prm[0] / 2), f = prm[1], l = prm[2];
        if (j == 0) {
            m[0] = -s / 2; m[1] = -cexp(I * l) * c / 2;
            m[2] = cexp(I * f) * c / 2; m[3] = -cexp(I * (f + l)) * s / 2;
        } else if (j == 1) {
            m[0] = 0; m[1] = 0; m[2] = I * cexp(I * f) * s; m[3] = I * cexp(I * (f + l)) * c;
        } else if (j == 2) {
            m[0] = 0; m[1] = -I * cexp(I * l) * s; m[2] = 0; m[3] = I * cexp(I * (f + l)) * c;
        } else {
            return -1;
        }
        return 1;
    }
    return -1;
}

/* ---------------------------------------------------------------- apply */

/* psi <- G(psi) for the gate (M, Q) with controls C. For every basis index
 * b whose target bits are all 0 and whose control bits are all 1, gather the
 * 2^k amplitudes idx(r) = b | sum_j bit(r, k-1-j) << Q[j], multiply by M,
 * scatter back. Other amplitudes are untouched. Returns 0, or -1 on bad
 * arguments. */
int orc_apply(cplx* psi, int n, int k, const int* tq, int nc, const int* cq, const cplx* m)
{
    if (k < 1 || k > ORC_MAX_K || n < k + nc || n > 40) return -1;
    uint64_t tmask = 0, cmask = 0;
    for (int j = 0; j < k; ++j) {
        if (tq[j] < 0 || tq[j] >= n || (tmask >> tq[j] & 1)) return -1;
        tmask |= 1ull << tq[j];
    }
    for (int j = 0; j < nc; ++j) {
        if (cq[j] < 0 || cq[j] >= n || ((tmask | cmask) >> cq[j] & 1)) return -1;
        cmask |= 1ull << cq[j];
    }
    const int64_t N = (int64_t)1 << n;
    const int d = 1 << k;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < N; ++b) {
        if ((uint64_t)b & tmask) continue;
        if (((uint64_t)b & cmask) != cmask) continue;
        uint64_t idx[1 << ORC_MAX_K];
        cplx v[1 << ORC_MAX_K], w[1 << ORC_MAX_K];
        for (int r = 0; r < d; ++r) {
            uint64_t a = (uint64_t)b;
            for (int j = 0; j < k; ++j)
                if ((r >> (k - 1 - j)) & 1) a |= 1ull << tq[j];
            idx[r] = a;
            v[r] = psi[a];
        }
        for (int r = 0; r < d; ++r) {
            cplx acc = 0;
            for (int s = 0; s < d; ++s) acc += m[r * d + s] * v[s];
            w[r] = acc;
        }
        for (int r = 0; r < d; ++r) psi[idx[r]] = w[r];
    }
    return 0;
}

/* Zero every amplitude whose control bits are not all 1 (the projector
 * onto the controlled subspace; used for derivatives of controlled gates). */
void orc_project_controls(cplx* psi, int n, int nc, const int* cq)
{
    uint64_t cmask = 0;
    for (int j = 0; j < nc; ++j) cmask |= 1ull << cq[j];
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < N; ++b)
        if (((uint64_t)b & cmask) != cmask) psi[b] = 0;
}

/* Zero every amplitude and set psi[idx] = 1 (the basis state e_idx). */
void orc_basis(cplx* psi, int n, uint64_t idx)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < N; ++b) psi[b] = 0;
    psi[idx] = 1;
}

/* ----------------------------------------------------------- reductions */

typedef struct { double s, c; } neum;

static void neum_add(neum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static double neum_val(const neum* a) { return a->s + a->c; }

#define ORC_CHUNKS 256

static inline int popc(uint64_t x) { return __builtin_popcountll(x); }

/* <P> for the Pauli string with x_mask (X or Y positions) and z_mask (Z or Y
 * positions): P = i^{|x&z|} X^x Z^z since Y = iXZ, so
 * <psi|P|psi> = sum_b conj(psi[b ^ x]) i^{|x&z|} (-1)^{|b&z|} psi[b].
 * Writes the real and imaginary parts (the latter is 0 up to rounding for a
 * Hermitian P). */
void orc_expval_pauli(const cplx* psi, int n, uint64_t xm, uint64_t zm, double* re, double* im)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t chunk = (N + ORC_CHUNKS - 1) / ORC_CHUNKS;
    neum pr[ORC_CHUNKS], pi[ORC_CHUNKS];
    cplx ph = 1;
    for (int j = 0; j < popc(xm & zm); ++j) ph *= I;
#pragma omp parallel for schedule(static)
    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
        neum ar = {0, 0}, ai = {0, 0};
        int64_t lo = ch * chunk, hi = lo + chunk < N ? lo + chunk : N;
        for (int64_t b = lo; b < hi; ++b) {
            double sg = (popc((uint64_t)b & zm) & 1) ? -1.0 : 1.0;
            cplx t = conj(psi[(uint64_t)b ^ xm]) * ph * sg * psi[b];
            neum_add(&ar, creal(t));
            neum_add(&ai, cimag(t));
        }
        pr[ch] = ar;
        pi[ch] = ai;
    }
    neum tr = {0, 0}, ti = {0, 0};
    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
        neum_add(&tr, neum_val(&pr[ch]));
        neum_add(&ti, neum_val(&pi[ch]));
    }
    *re = neum_val(&tr);
    *im = neum_val(&ti);
}

/* <Z_i> = sum_b |psi_b|^2 (1 - 2 b_i) for every qubit i, written to out[i],
 * and ||psi||^2 = sum_b |psi_b|^2 written to out[n]. */
void orc_expval_z_all(const cplx* psi, int n, double* out)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t chunk = (N + ORC_CHUNKS - 1) / ORC_CHUNKS;
    static neum part[ORC_CHUNKS][65];
#pragma omp parallel for schedule(static)
    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
        neum acc[65];
        memset(acc, 0, sizeof(acc));
        int64_t lo = ch * chunk, hi = lo + chunk < N ? lo + chunk : N;
        for (int64_t b = lo; b < hi; ++b) {
            double pb = creal(psi[b]) * creal(psi[b]) + cimag(psi[b]) * cimag(psi[b]);
            for (int i = 0; i < n; ++i) neum_add(&acc[i], ((b >> i) & 1) ? -pb : pb);
            neum_add(&acc[n], pb);
        }
        memcpy(part[ch], acc, sizeof(acc));
    }
    for (int i = 0; i <= n; ++i) {
        neum t = {0, 0};
        for (int ch = 0; ch < ORC_CHUNKS; ++ch) neum_add(&t, neum_val(&part[ch][i]));
        out[i] = neum_val(&t);
    }
}

/* <a|b> = sum_i conj(a_i) b_i, real and imaginary parts. */
void orc_inner(const cplx* a, const cplx* b, int n, double* re, double* im)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t chunk = (N + ORC_CHUNKS - 1) / ORC_CHUNKS;
    neum pr[ORC_CHUNKS], pi[ORC_CHUNKS];
#pragma omp parallel for schedule(static)
    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
        neum ar = {0, 0}, ai = {0, 0};
        int64_t lo = ch * chunk, hi = lo + chunk < N ? lo + chunk : N;
        for (int64_t i = lo; i < hi; ++i) {
            cplx t = conj(a[i]) * b[i];
            neum_add(&ar, creal(t));
            neum_add(&ai, cimag(t));
        }
        pr[ch] = ar;
        pi[ch] = ai;
    }
    neum tr = {0, 0}, ti = {0, 0};
    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
        neum_add(&tr, neum_val(&pr[ch]));
        neum_add(&ti, neum_val(&pi[ch]));
    }
    *re = neum_val(&tr);
    *im = neum_val(&ti);
}

/* out <- sum_t coeff_t P_t psi for Pauli strings (x_mask, z_mask) (the
 * observable applied to the state; the start of the adjoint recursion). */
void orc_apply_pauli_sum(const cplx* psi, int n, int nt, const uint64_t* xm, const uint64_t* zm,
                         const double* coeff, cplx* out)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < N; ++b) {
        /* (P psi)[b ^ x] = i^{|x&z|} (-1)^{|b&z|} psi[b]  <=>
         * (P psi)[c] = i^{|x&z|} (-1)^{|(c^x)&z|} psi[c ^ x] */
        cplx acc = 0;
        for (int t = 0; t < nt; ++t) {
            cplx ph = 1;
            for (int j = 0; j < popc(xm[t] & zm[t]); ++j) ph *= I;
            uint64_t src = (uint64_t)b ^ xm[t];
            double sg = (popc(src & zm[t]) & 1) ? -1.0 : 1.0;
            acc += coeff[t] * ph * sg * psi[src];
        }
        out[b] = acc;
    }
}

/* ---------------------------------------------------------------- shots */

/* Running sum of the Z-basis probabilities (Sec. 2.2.1): cdf[b] =
 * sum_{c <= b} |psi_c|^2, one Neumaier-compensated sum in index order. */
void orc_prob_cdf(const cplx* psi, int n, double* cdf)
{
    const int64_t N = (int64_t)1 << n;
    neum a = {0, 0};
    for (int64_t b = 0; b < N; ++b) {
        const double re = creal(psi[b]), im = cimag(psi[b]);
        neum_add(&a, re * re + im * im);
        cdf[b] = neum_val(&a);
    }
}

/* Exact shot sampling (Sec. 4.3.1): each shot s is a draw of the basis index
 * b with probability p_b = |psi_b|^2 / T, T = cdf[N-1], by inverse CDF: the
 * smallest b with cdf[b] > t_s, t_s = u_s T clamped below T (so a u_s that
 * rounds up to T takes the last index of non-zero probability). The counts
 * of the returned indices over the shots are one draw of the multinomial
 * M(shots, p). A state of zero norm returns -1 for every shot. */
void orc_sample_exact(const double* cdf, int n, const double* u, int64_t shots, int64_t* out)
{
    const int64_t N = (int64_t)1 << n;
    const double T = cdf[N - 1];
    for (int64_t s = 0; s < shots; ++s) {
        double t = u[s] * T;
        if (t >= T) t = nextafter(T, 0.0);
        /* binary search for the first cdf > t */
        int64_t lo = 0, hi = N;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > t) hi = mid;
            else lo = mid + 1;
        }
        out[s] = lo < N ? lo : -1;
    }
}

/* Gaussian approximation of the shot histogram (Sec. 4.3.2), as the
 * reparameterised draw y = shots p + sqrt(shots) D S z with
 *   p = |psi|^2 / T, u = sqrt(p), D = diag(u),
 *   v = (e - u) / ||e - u||, e the last basis vector (v = 0 when u = e),
 *   S = I - 2 v v^T (the Householder reflection that maps e to u),
 *   z = (z_0, ..., z_{N-2}, 0).
 * S z is applied as z - 2 v (v . z). Sums are Neumaier-compensated. */
void orc_sample_gaussian(const cplx* psi, int n, const double* z, double shots, double* y)
{
    const int64_t N = (int64_t)1 << n;
    neum tn = {0, 0};
    for (int64_t b = 0; b < N; ++b) {
        const double re = creal(psi[b]), im = cimag(psi[b]);
        neum_add(&tn, re * re + im * im);
    }
    const double T = neum_val(&tn);
    /* ||e - u||^2 and v . z (z_last = 0) */
    neum r2 = {0, 0}, vz = {0, 0};
    for (int64_t b = 0; b < N; ++b) {
        const double re = creal(psi[b]), im = cimag(psi[b]);
        const double u = sqrt((re * re + im * im) / T);
        const double d = (b == N - 1 ? 1.0 : 0.0) - u;
        neum_add(&r2, d * d);
        if (b < N - 1) neum_add(&vz, d * z[b]);
    }
    const double r = sqrt(neum_val(&r2));
    const double vdotz = r > 0 ? neum_val(&vz) / r : 0.0;
    for (int64_t b = 0; b < N; ++b) {
        const double re = creal(psi[b]), im = cimag(psi[b]);
        const double p = (re * re + im * im) / T;
        const double u = sqrt(p);
        const double v = r > 0 ? ((b == N - 1 ? 1.0 : 0.0) - u) / r : 0.0;
        const double zb = b < N - 1 ? z[b] : 0.0;
        y[b] = shots * p + sqrt(shots) * u * (zb - 2.0 * v * vdotz);
    }
}

/* Gaussian estimate of every <Z_i> (Sec. 4.3.2): the histogram y of
 * orc_sample_gaussian turned into E_i = (1/shots) sum_b y_b s_i(b) with
 * s_i(b) = 1 - 2 (bit i of b), i.e. the Z_i eigenvalue of b. */
void orc_gaussian_z(const cplx* psi, int n, const double* z, double shots, double* est, double* y_work)
{
    const int64_t N = (int64_t)1 << n;
    orc_sample_gaussian(psi, n, z, shots, y_work);
    for (int i = 0; i < n; ++i) {
        neum a = {0, 0};
        for (int64_t b = 0; b < N; ++b) neum_add(&a, ((b >> i) & 1) ? -y_work[b] : y_work[b]);
        est[i] = neum_val(&a) / shots;
    }
}

/* Derivative of F = sum_i g_i E_i with respect to the unnormalised
 * probabilities q_b = |psi_b|^2, for fixed normals z (the reparameterised
 * estimate of Sec. 4.3.2 is a smooth function of q). With T = sum q,
 * p = q / T, u = sqrt p, d = e - u (e the last basis vector), R = ||d||^2,
 * K = d . z, c_b = sum_i g_i s_i(b), Q = sum_b c_b u_b d_b:
 *   F = sum_b c_b p_b + (1/sqrt shots) sum_b c_b u_b (S z)_b,
 *   (S z)_b = z_b - 2 d_b K / R,
 *   dF/dp_b = c_b + c_b K / (R sqrt shots)
 *             + (c_b (S z)_b + 2 z_b Q / R - 4 d_b K Q / R^2) / (2 u_b sqrt shots)
 *   (the last term taken as 0 where u_b = 0: the square root has no
 *   derivative at 0), and dF/dq_b = (dF/dp_b - sum_b' p_b' dF/dp_b') / T. */
void orc_gaussian_z_weights(const cplx* psi, int n, const double* z, double shots, const double* g, double* w)
{
    const int64_t N = (int64_t)1 << n;
    neum tn = {0, 0};
    for (int64_t b = 0; b < N; ++b) {
        const double re = creal(psi[b]), im = cimag(psi[b]);
        neum_add(&tn, re * re + im * im);
    }
    const double T = neum_val(&tn);
    const double sq = sqrt(shots);
    neum rn = {0, 0}, kn = {0, 0}, qn = {0, 0};
    for (int64_t b = 0; b < N; ++b) {
        const double re = creal(psi[b]), im = cimag(psi[b]);
        const double u = sqrt((re * re + im * im) / T);
        const double d = (b == N - 1 ? 1.0 : 0.0) - u;
        const double zb = b < N - 1 ? z[b] : 0.0;
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += ((b >> i) & 1) ? -g[i] : g[i];
        neum_add(&rn, d * d);
        neum_add(&kn, d * zb);
        neum_add(&qn, c * u * d);
    }
    const double R = neum_val(&rn), K = neum_val(&kn), Q = neum_val(&qn);
    neum mn = {0, 0};
    for (int64_t b = 0; b < N; ++b) {
        const double re = creal(psi[b]), im = cimag(psi[b]);
        const double p = (re * re + im * im) / T;
        const double u = sqrt(p);
        const double d = (b == N - 1 ? 1.0 : 0.0) - u;
        const double zb = b < N - 1 ? z[b] : 0.0;
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += ((b >> i) & 1) ? -g[i] : g[i];
        double wp = c;
        if (R > 0.0) {
            const double sz = zb - 2.0 * d * K / R;
            wp += c * K / (R * sq);
            if (u > 0.0) wp += (c * sz + 2.0 * zb * Q / R - 4.0 * d * K * Q / (R * R)) / (2.0 * u * sq);
        } else if (u > 0.0) {
            wp += c * zb / (2.0 * u * sq);   /* S = I when u = e */
        }
        w[b] = wp;
        neum_add(&mn, p * wp);
    }
    const double M = neum_val(&mn);
    for (int64_t b = 0; b < N; ++b) w[b] = (w[b] - M) / T;
}
