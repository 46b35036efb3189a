// gatemath.cpp -- complex128 matrices of the named gate kinds and their
// parameter derivatives (host side of the GPU library).
//
// Rotations: R_P(t) = exp(-i t P / 2); because P^2 = I this is
// cos(t/2) I - i sin(t/2) P (the single-qubit Pauli rotations of Sec. 3,
// and their two-qubit P(x)P forms). U3 is the OpenQASM 2 gate; P(l) is the
// phase gate diag(1, e^{il}). Index order: first target = most significant
// bit of the matrix index (Sec. 4.1.1, MoveDim moves Q to the front).
#include <cmath>
#include <cstring>

#include "sv_internal.h"

namespace sv {

namespace {

const cd kI(0.0, 1.0);

// Pauli matrices, 2x2 row-major.
void pauli2(char p, cd* out)
{
    static const cd X[4] = {0.0, 1.0, 1.0, 0.0};
    static const cd Y[4] = {0.0, cd(0, -1), cd(0, 1), 0.0};
    static const cd Z[4] = {1.0, 0.0, 0.0, -1.0};
    const cd* src = p == 'x' ? X : p == 'y' ? Y : Z;
    for (int i = 0; i < 4; ++i) out[i] = src[i];
}

// Generator P of a rotation kind; returns its qubit count, 0 if not a rotation.
int rotation_generator(int kind, cd* P)
{
    char axis;
    int k;
    switch (kind) {
    case SV_RX: axis = 'x'; k = 1; break;
    case SV_RY: axis = 'y'; k = 1; break;
    case SV_RZ: axis = 'z'; k = 1; break;
    case SV_RXX: axis = 'x'; k = 2; break;
    case SV_RYY: axis = 'y'; k = 2; break;
    case SV_RZZ: axis = 'z'; k = 2; break;
    default: return 0;
    }
    cd p[4];
    pauli2(axis, p);
    if (k == 1) {
        std::memcpy(P, p, sizeof(p));
        return 1;
    }
    // P (x) P, row (a1 a0), col (b1 b0) -> p[a1][b1] * p[a0][b0]
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) P[a * 4 + b] = p[(a >> 1) * 2 + (b >> 1)] * p[(a & 1) * 2 + (b & 1)];
    return 2;
}

}  // namespace

int kind_targets(int kind)
{
    switch (kind) {
    case SV_SWAP: case SV_RXX: case SV_RYY: case SV_RZZ: return 2;
    case SV_MATRIX: return 0;
    default: return (kind >= SV_H && kind <= SV_U3) ? 1 : -1;
    }
}

int kind_nparams(int kind)
{
    switch (kind) {
    case SV_RX: case SV_RY: case SV_RZ: case SV_P: case SV_RXX: case SV_RYY: case SV_RZZ: return 1;
    case SV_U3: return 3;
    default: return 0;
    }
}

int kind_matrix(int kind, const double* prm, cd* m)
{
    cd P[16];
    if (int k = rotation_generator(kind, P)) {
        const int d = 1 << k;
        const double c = std::cos(0.5 * prm[0]), s = std::sin(0.5 * prm[0]);
        for (int r = 0; r < d; ++r)
            for (int q = 0; q < d; ++q) m[r * d + q] = (r == q ? cd(c) : cd(0.0)) - kI * s * P[r * d + q];
        return k;
    }
    const double h = 1.0 / std::sqrt(2.0);
    auto set2 = [&](cd a, cd b, cd c, cd d) { m[0] = a; m[1] = b; m[2] = c; m[3] = d; return 1; };
    switch (kind) {
    case SV_H: return set2(h, h, h, -h);
    case SV_X: return set2(0.0, 1.0, 1.0, 0.0);
    case SV_Y: return set2(0.0, -kI, kI, 0.0);
    case SV_Z: return set2(1.0, 0.0, 0.0, -1.0);
    case SV_S: return set2(1.0, 0.0, 0.0, kI);
    case SV_SDG: return set2(1.0, 0.0, 0.0, -kI);
    case SV_T: return set2(1.0, 0.0, 0.0, std::polar(1.0, M_PI / 4));
    case SV_TDG: return set2(1.0, 0.0, 0.0, std::polar(1.0, -M_PI / 4));
    case SV_SX: return set2(cd(0.5, 0.5), cd(0.5, -0.5), cd(0.5, -0.5), cd(0.5, 0.5));
    case SV_P: return set2(1.0, 0.0, 0.0, std::polar(1.0, prm[0]));
    case SV_U3: {
        const double c = std::cos(0.5 * prm[0]), s = std::sin(0.5 * prm[0]);
        return set2(c, -std::polar(s, prm[2]), std::polar(s, prm[1]), std::polar(c, prm[1] + prm[2]));
    }
    case SV_SWAP:
        for (int i = 0; i < 16; ++i) m[i] = 0.0;
        m[0] = m[15] = 1.0;
        m[1 * 4 + 2] = m[2 * 4 + 1] = 1.0;
        return 2;
    default: return -1;
    }
}

int kind_dmatrix(int kind, const double* prm, int j, cd* m)
{
    cd P[16];
    if (int k = rotation_generator(kind, P)) {
        if (j != 0) return -1;
        const int d = 1 << k;
        const double dc = -0.5 * std::sin(0.5 * prm[0]), ds = 0.5 * std::cos(0.5 * prm[0]);
        for (int r = 0; r < d; ++r)
            for (int q = 0; q < d; ++q) m[r * d + q] = (r == q ? cd(dc) : cd(0.0)) - kI * ds * P[r * d + q];
        return k;
    }
    if (kind == SV_P) {
        if (j != 0) return -1;
        m[0] = m[1] = m[2] = 0.0;
        m[3] = kI * std::polar(1.0, prm[0]);
        return 1;
    }
    if (kind == SV_U3) {
        const double c = std::cos(0.5 * prm[0]), s = std::sin(0.5 * prm[0]);
        const double f = prm[1], l = prm[2];
        switch (j) {
        case 0:  // d/dtheta
            m[0] = -0.5 * s;
            m[1] = -std::polar(0.5 * c, l);
            m[2] = std::polar(0.5 * c, f);
            m[3] = -std::polar(0.5 * s, f + l);
            return 1;
        case 1:  // d/dphi
            m[0] = m[1] = 0.0;
            m[2] = kI * std::polar(s, f);
            m[3] = kI * std::polar(c, f + l);
            return 1;
        case 2:  // d/dlambda
            m[0] = m[2] = 0.0;
            m[1] = -kI * std::polar(s, l);
            m[3] = kI * std::polar(c, f + l);
            return 1;
        default: return -1;
        }
    }
    return -1;
}

}  // namespace sv
