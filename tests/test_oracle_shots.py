"""Pins of the oracle's shot sampling (Sec. 4.3), CPU only.

Exact sampling: a hand-worked example (tests/golden/shots_worked_example.json),
the library routine of the same definition (numpy searchsorted over a
cumulative sum), zero-probability indices never drawn, clamping at u -> 1, a
zero state, and a chi-square test of 400 000 draws against p.

Gaussian approximation (Sec. 4.3.2, with the readings: S = I - 2 v v^T, e the
last basis vector, z_last = 0): the reflection's algebra checked with an
explicit matrix (S e = u, S^2 = I, D S (I - e e^T) S D = diag p - p p^T, the
multinomial covariance), the oracle's draw equal to the explicit matrix
formula, sum(y) = shots, point masses giving no noise, and the sample mean and
covariance of 40 000 draws against shots p and shots (diag p - p p^T).
"""

import json
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from tests import pins

HERE = os.path.dirname(os.path.abspath(__file__))


def _state_from_probs(p, rng=None):
    p = np.asarray(p, dtype=np.float64)
    ph = np.ones(len(p)) if rng is None else np.exp(2j * np.pi * rng.random(len(p)))
    return np.sqrt(p) * ph


def test_exact_worked_example():
    g = json.load(open(os.path.join(HERE, "golden", "shots_worked_example.json")))
    psi = _state_from_probs(g["probabilities"], np.random.default_rng(1))
    got = oracle.sample_exact(psi, 3, np.array(g["uniforms"]))
    assert got.tolist() == g["indices"]


@pytest.mark.parametrize("n,seed", [(1, 1), (4, 2), (9, 3), (14, 4)])
def test_exact_matches_searchsorted(n, seed):
    rng = np.random.default_rng(seed)
    psi = pins.random_state(n, rng)
    u = rng.random(5000)
    got = oracle.sample_exact(psi, n, u)
    p = np.abs(psi) ** 2
    c = np.cumsum(p)
    want = np.searchsorted(c, u * c[-1], side="right")
    # away from the CDF steps (rounding of two summation orders) the two agree
    far = np.min(np.abs(c[np.clip(want, 0, len(c) - 1)][:, None] - (u * c[-1])[:, None]), axis=1) > 1e-12
    assert np.array_equal(got[far], want[far])
    assert np.all((got >= 0) & (got < (1 << n)))


def test_exact_never_draws_zero_probability():
    rng = np.random.default_rng(7)
    p = rng.random(64)
    p[rng.random(64) < 0.5] = 0.0
    p[0] = 0.0                      # u = 0 must not return index 0
    p /= p.sum()
    psi = _state_from_probs(p, rng)
    u = np.concatenate([[0.0], rng.random(20000), [np.nextafter(1.0, 0.0)]])
    got = oracle.sample_exact(psi, 6, u)
    assert np.all(p[got] > 0)
    assert got[0] == np.flatnonzero(p)[0]
    assert got[-1] == np.flatnonzero(p)[-1]          # clamped below T: the last non-zero index


def test_exact_basis_and_zero_state():
    psi = np.zeros(16, dtype=np.complex128)
    psi[11] = 1j
    assert np.all(oracle.sample_exact(psi, 4, np.linspace(0, 0.999, 50)) == 11)
    assert np.all(oracle.sample_exact(np.zeros(16, dtype=np.complex128), 4, np.array([0.0, 0.5])) == -1)


def test_exact_chi_square():
    rng = np.random.default_rng(11)
    psi = pins.random_state(4, rng)
    p = np.abs(psi) ** 2
    p /= p.sum()
    shots = 400_000
    got = oracle.sample_exact(psi, 4, rng.random(shots))
    counts = np.bincount(got, minlength=16)
    chi2 = np.sum((counts - shots * p) ** 2 / (shots * p))
    assert chi2 < stats.chi2.ppf(1 - 1e-6, 15)


def _reflection(p):
    u = np.sqrt(p)
    e = np.zeros(len(p))
    e[-1] = 1.0
    vt = e - u
    nv = np.linalg.norm(vt)
    v = vt / nv if nv > 0 else np.zeros(len(p))
    return np.eye(len(p)) - 2.0 * np.outer(v, v), u, e


def test_gaussian_reflection_algebra():
    rng = np.random.default_rng(5)
    p = rng.random(8)
    p /= p.sum()
    S, u, e = _reflection(p)
    np.testing.assert_allclose(S, S.T, atol=1e-15)
    np.testing.assert_allclose(S @ S, np.eye(8), atol=1e-14)
    np.testing.assert_allclose(S @ e, u, atol=1e-14)
    D = np.diag(u)
    cov = D @ S @ (np.eye(8) - np.outer(e, e)) @ S.T @ D
    np.testing.assert_allclose(cov, np.diag(p) - np.outer(p, p), atol=1e-14)


@pytest.mark.parametrize("n,seed", [(1, 1), (3, 2), (6, 3)])
def test_gaussian_matches_explicit_matrix(n, seed):
    rng = np.random.default_rng(seed)
    psi = pins.random_state(n, rng) * 1.3          # an unnormalised state: p is normalised
    z = rng.normal(size=1 << n)
    shots = 2500.0
    y = oracle.sample_gaussian(psi, n, z, shots)
    p = np.abs(psi) ** 2
    p /= p.sum()
    S, u, _ = _reflection(p)
    zz = z.copy()
    zz[-1] = 0.0
    want = shots * p + np.sqrt(shots) * np.diag(u) @ S @ zz
    np.testing.assert_allclose(y, want, rtol=1e-12, atol=1e-9)
    assert abs(y.sum() - shots) < 1e-9 * shots


def test_gaussian_point_masses_have_no_noise():
    z = np.random.default_rng(3).normal(size=8)
    for idx in (0, 3, 7):
        psi = np.zeros(8, dtype=np.complex128)
        psi[idx] = np.exp(0.4j)
        y = oracle.sample_gaussian(psi, 3, z, 1000.0)
        want = np.zeros(8)
        want[idx] = 1000.0
        np.testing.assert_allclose(y, want, atol=1e-10)


def test_gaussian_moments_match_multinomial():
    rng = np.random.default_rng(9)
    psi = pins.random_state(3, rng)
    p = np.abs(psi) ** 2
    p /= p.sum()
    shots = 500.0
    draws = np.array([oracle.sample_gaussian(psi, 3, rng.normal(size=8), shots) for _ in range(40000)])
    mean = draws.mean(axis=0)
    cov = np.cov(draws.T)
    want_cov = shots * (np.diag(p) - np.outer(p, p))
    sd = np.sqrt(np.diag(want_cov))
    assert np.all(np.abs(mean - shots * p) < 5 * sd / np.sqrt(40000) + 1e-9)
    assert np.max(np.abs(cov - want_cov)) < 0.05 * shots * p.max()


# ---- the differentiable Gaussian estimate of every <Z_i> (Sec. 4.3.2 with
# the normals held fixed: a smooth function of the probabilities)

def test_gaussian_z_without_noise_is_the_exact_expectation():
    """z = 0: y = shots p, so E_i is <Z_i> itself (the plain definition)."""
    rng = np.random.default_rng(4)
    n = 6
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    est = oracle.gaussian_z(psi, n, np.zeros(1 << n), 500.0)
    want = [np.sum(np.abs(psi) ** 2 * (1 - 2 * ((np.arange(1 << n) >> i) & 1))) for i in range(n)]
    np.testing.assert_allclose(est, want, atol=1e-14)


def test_gaussian_z_is_the_histogram_read_out():
    """E_i = (1/shots) sum_b y_b s_i(b) over the sampler's histogram."""
    rng = np.random.default_rng(5)
    n = 5
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    z = rng.normal(size=1 << n)
    y = oracle.sample_gaussian(psi, n, z, 800.0)
    sign = 1 - 2 * ((np.arange(1 << n)[:, None] >> np.arange(n)) & 1)
    np.testing.assert_allclose(oracle.gaussian_z(psi, n, z, 800.0), y @ sign / 800.0, atol=1e-12)


@pytest.mark.parametrize("n,seed,shots", [(4, 1, 100.0), (5, 2, 1000.0), (6, 3, 1e5)])
def test_gaussian_z_weights_are_the_derivative(n, seed, shots):
    """The weights w_b = dF/d|psi_b|^2 (F = sum_i g_i E_i) against central
    differences of the oracle's own estimate: |psi_b|^2 moved by +-h with the
    phase kept (the step error is O(h^2); h = 1e-7)."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    psi = rng.normal(size=N) + 1j * rng.normal(size=N)
    psi /= np.linalg.norm(psi)
    z = rng.normal(size=N)
    g = rng.normal(size=n)
    w = oracle.gaussian_z_weights(psi, n, z, shots, g)

    def F(ps):
        return float(np.dot(g, oracle.gaussian_z(ps, n, z, shots)))

    h = 1e-7
    for b in range(N):
        q = abs(psi[b]) ** 2
        pp, pm = psi.copy(), psi.copy()
        pp[b] *= np.sqrt((q + h) / q)
        pm[b] *= np.sqrt((q - h) / q)
        fd = (F(pp) - F(pm)) / (2 * h)
        assert abs(fd - w[b]) < 1e-6 * max(1.0, abs(w[b])), (b, fd, w[b])


def test_gaussian_z_weights_without_noise():
    """z = 0: F = sum_b c_b p_b with p = q / T, so w_b = (c_b - F) / T with
    c_b = sum_i g_i s_i(b) (T = 1 here)."""
    rng = np.random.default_rng(6)
    n = 5
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    g = rng.normal(size=n)
    sign = 1 - 2 * ((np.arange(1 << n)[:, None] >> np.arange(n)) & 1)
    c = sign @ g
    F = float(np.sum(np.abs(psi) ** 2 * c))
    w = oracle.gaussian_z_weights(psi, n, np.zeros(1 << n), 300.0, g)
    np.testing.assert_allclose(w, c - F, atol=1e-12)
