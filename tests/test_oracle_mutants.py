"""The oracle's pins have teeth: plausible mistakes planted in a copy of the
oracle's C source (on the CPU) each make at least one independent pin fail.

Each mutant is compiled into a temporary library and run through a compact
set of pin checks (Kronecker / Alg. 1 brute force, closed forms, Pauli
expectations against dense operators, gradient cross-checks)."""

import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from oracle import build as obuild
from paper_2511_19291_amd import circuits as C
from tests import pins

MUTANTS = {
    "target bit order": ("if ((r >> (k - 1 - j)) & 1) a |= 1ull << tq[j];", "if ((r >> j) & 1) a |= 1ull << tq[j];"),
    "transposed matrix": ("acc += m[r * d + s] * v[s];", "acc += m[s * d + r] * v[s];"),
    "u3 sign": ("m[1] = -cexp(I * l) * s;", "m[1] = cexp(I * l) * s;"),
    "rotation half angle": ("double c = cos(prm[0] / 2), s = sin(prm[0] / 2);\n        for (int r = 0; r < d; ++r)",
                            "double c = cos(prm[0]), s = sin(prm[0]);\n        for (int r = 0; r < d; ++r)"),
    "rotation sign": ("m[r * d + q] = (r == q ? c : 0.0) - I * s * p[r * d + q];",
                      "m[r * d + q] = (r == q ? c : 0.0) + I * s * p[r * d + q];"),
    "controls ignored": ("if (((uint64_t)b & cmask) != cmask) continue;\n        uint64_t idx", "uint64_t idx"),
    "pauli z sign mask": ("double sg = (popc((uint64_t)b & zm) & 1) ? -1.0 : 1.0;",
                          "double sg = (popc((uint64_t)b & xm) & 1) ? -1.0 : 1.0;"),
    "Y phase dropped": ("for (int j = 0; j < popc(xm & zm); ++j) ph *= I;\n#pragma omp parallel for schedule(static)\n    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {\n        neum ar",
                        "#pragma omp parallel for schedule(static)\n    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {\n        neum ar"),
    "z_all bit test": ("neum_add(&acc[i], ((b >> i) & 1) ? -pb : pb);", "neum_add(&acc[i], ((b >> (n - 1 - i)) & 1) ? -pb : pb);"),
    "derivative scale": ("double dc = -0.5 * sin(prm[0] / 2), ds = 0.5 * cos(prm[0] / 2);",
                         "double dc = -sin(prm[0] / 2), ds = cos(prm[0] / 2);"),
    "cdf tie rule": ("if (cdf[mid] > t) hi = mid;", "if (cdf[mid] >= t) hi = mid;"),
    "householder factor": ("y[b] = shots * p + sqrt(shots) * u * (zb - 2.0 * v * vdotz);",
                           "y[b] = shots * p + sqrt(shots) * u * (zb - v * vdotz);"),
    "reflection target": ("const double v = r > 0 ? ((b == N - 1 ? 1.0 : 0.0) - u) / r : 0.0;",
                          "const double v = r > 0 ? ((b == 0 ? 1.0 : 0.0) - u) / r : 0.0;"),
    "last normal kept": ("const double zb = b < N - 1 ? z[b] : 0.0;", "const double zb = z[b];"),
    "weights reflection sign": ("- 4.0 * d * K * Q / (R * R)) / (2.0 * u * sq);",
                                "+ 4.0 * d * K * Q / (R * R)) / (2.0 * u * sq);"),
    "weights normalisation dropped": ("for (int64_t b = 0; b < N; ++b) w[b] = (w[b] - M) / T;",
                                      "for (int64_t b = 0; b < N; ++b) w[b] = w[b] / T;"),
    "weights sqrt derivative": ("Q / (R * R)) / (2.0 * u * sq);", "Q / (R * R)) / (u * sq);"),
}


def _pins_pass() -> bool:
    """A compact set of the independent pins; False as soon as one fails."""
    rng = np.random.default_rng(5)
    try:
        for n, seed in [(3, 1), (5, 2)]:
            circ = C.random_circuit(n, 40, seed)
            psi = oracle.run(circ)
            u = np.eye(1 << n, dtype=np.complex128)
            for op in circ.ops:
                m = pins.textbook_matrix(op.kind, [circ.params[i] for i in op.params])
                u = pins.embed_kron(m, n, op.targets, op.controls) @ u
            if np.max(np.abs(psi - u[:, 0])) > 1e-12:
                return False
        # an asymmetric dense matrix on unsorted targets (the named 2-qubit
        # kinds are symmetric under exchanging their qubits)
        n, targets = 5, [3, 0, 4]
        m = pins.haar_unitary(8, rng)
        psi0 = pins.random_state(n, rng)
        psi = psi0.copy()
        oracle.apply_matrix(psi, n, m, targets)
        if np.max(np.abs(psi - pins.embed_kron(m, n, targets) @ psi0)) > 1e-12:
            return False
        n = 4
        psi = pins.random_state(n, rng)
        for _ in range(10):
            xm, zm = int(rng.integers(0, 16)), int(rng.integers(0, 16))
            ref = psi.conj() @ pins.pauli_matrix(n, xm, zm) @ psi
            if abs(oracle.expval_pauli(psi, n, xm, zm)[0] - ref.real) > 1e-12:
                return False
        z, _ = oracle.expval_z_all(psi, n)
        p = np.abs(psi) ** 2
        b = np.arange(1 << n)
        if any(abs(z[i] - np.sum(p * (1 - 2 * ((b >> i) & 1)))) > 1e-12 for i in range(n)):
            return False
        # shots: exact draws vs the library routine of the definition (with a
        # zero-probability first index and u = 0), the Gaussian draw vs the
        # explicit reflection matrix
        pz = np.abs(psi) ** 2
        pz[0] = 0.0
        psz = np.sqrt(pz)
        us = np.concatenate([[0.0], rng.random(200)])
        cs = np.cumsum(pz)
        if not np.array_equal(oracle.sample_exact(psz, n, us), np.searchsorted(cs, us * cs[-1], side="right")):
            return False
        zs = rng.normal(size=1 << n)
        pp = pz / pz.sum()
        uu = np.sqrt(pp)
        e = np.zeros(1 << n)
        e[-1] = 1.0
        vv = (e - uu) / np.linalg.norm(e - uu)
        zz = zs.copy()
        zz[-1] = 0.0
        want = 100.0 * pp + 10.0 * uu * ((np.eye(1 << n) - 2 * np.outer(vv, vv)) @ zz)
        if np.max(np.abs(oracle.sample_gaussian(psz, n, zs, 100.0) - want)) > 1e-9:
            return False
        # the Gaussian estimate's weights vs central differences of the estimate
        gz = rng.normal(size=n)
        wz = oracle.gaussian_z_weights(psi, n, zs, 50.0, gz)
        for b in range(1 << n):
            q = abs(psi[b]) ** 2
            pp, pm = psi.copy(), psi.copy()
            pp[b] *= np.sqrt((q + 1e-7) / q)
            pm[b] *= np.sqrt((q - 1e-7) / q)
            fd = (np.dot(gz, oracle.gaussian_z(pp, n, zs, 50.0)) - np.dot(gz, oracle.gaussian_z(pm, n, zs, 50.0))) / 2e-7
            if abs(fd - wz[b]) > 1e-5 * max(1.0, abs(wz[b])):
                return False
        circ = C.rxry_ring(4, 2, 8)
        terms = C.z_sum_terms(4)
        g_fd = oracle.grad_finite_diff(circ, terms, h=1e-4)
        _, g_adj, _ = oracle.grad_adjoint(circ, terms)
        if np.max(np.abs(g_adj - g_fd)) > 1e-6:
            return False
        return True
    except ValueError:
        return False


def test_unmutated_oracle_passes_the_compact_pins():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    old, new = MUTANTS[name]
    src = open(obuild.SRC).read()
    assert old in src, f"mutation site for {name!r} not found"
    with tempfile.TemporaryDirectory() as d:
        csrc = os.path.join(d, "mutant.c")
        lib = os.path.join(d, "libmutant.so")
        with open(csrc, "w") as f:
            f.write(src.replace(old, new, 1))
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", lib, csrc, "-lm"],
                       check=True, capture_output=True)
        with oracle.using_library(lib):
            assert not _pins_pass(), f"mutant {name!r} passed every pin"
