"""GPU parity of shot sampling (Sec. 4.3) against the oracle, through the C ABI.

Exact sampling: the GPU and the oracle get the same complex64 amplitudes and
the same uniforms. Indices are integers decided by FP64 running sums that the
two sides add up in different orders, so they must be equal except where a
uniform lies within rounding distance (1e-12 relative) of a CDF step; there
the GPU's index must still be valid for the oracle's CDF within that
distance. Edge cases: u = 0 and u -> 1, zero-probability indices (never
drawn), a zero state (-1), no shots, determinism, a chi-square test of 2^20
draws, full-size 30-qubit states checked by properties (GHZ: only the two
non-zero indices, half each; a product state: independent bits with the
closed-form marginals).

Gaussian approximation: the GPU's y against the oracle's elementwise (FP64 on
both sides from the same inputs: rtol 1e-9), point masses, sum(y) = shots,
and at 30 qubits the noise energy sum (y - shots p)^2 / shots against its
expectation 1 - sum p^2.
"""

import numpy as np
import pytest

import oracle
from paper_2511_19291_amd import circuits as C
from paper_2511_19291_amd import sv as svmod
from tests import pins

pytestmark = pytest.mark.gpu

EPS = 1e-12


def _upload(sv, psi64):
    n = int(np.log2(len(psi64)))
    st = sv.State(n).from_numpy(psi64.astype(np.complex64)[None, :])
    return st, psi64.astype(np.complex64).astype(np.complex128)


def _check_exact(got, psi, n, u):
    want = oracle.sample_exact(psi, n, u)
    cdf = oracle.prob_cdf(psi, n)
    T = cdf[-1]
    t = np.minimum(u * T, np.nextafter(T, 0.0))
    bad = np.flatnonzero(got != want)
    for s in bad:
        g = got[s]
        assert 0 <= g < (1 << n), (s, g)
        lo = cdf[g - 1] if g > 0 else 0.0
        # valid within rounding distance of a step
        assert lo <= t[s] + EPS * T and cdf[g] > t[s] - EPS * T, (s, g, want[s])
    assert len(bad) <= max(2, len(u) // 10000), f"{len(bad)} of {len(u)} draws differ"


@pytest.mark.parametrize("n,seed", [(1, 1), (3, 2), (8, 3), (12, 4), (13, 5), (17, 6), (20, 7)])
def test_exact_parity(sv, n, seed):
    rng = np.random.default_rng(seed)
    st, psi = _upload(sv, pins.random_state(n, rng))
    u = np.concatenate([[0.0, np.nextafter(1.0, 0.0)], rng.random(20000)])
    got = st.sample_exact(u).cpu().numpy()
    _check_exact(got, psi, n, u)


def test_exact_sparse_states_never_draw_zero_probability(sv):
    rng = np.random.default_rng(8)
    n = 14
    p = rng.random(1 << n)
    p[rng.random(1 << n) < 0.97] = 0.0
    p[:5000] = 0.0                          # whole empty blocks, and u = 0 lands after them
    psi = np.sqrt(p / p.sum()) * np.exp(2j * np.pi * rng.random(1 << n))
    st, psi = _upload(sv, psi)
    u = np.concatenate([[0.0, np.nextafter(1.0, 0.0)], rng.random(50000)])
    got = st.sample_exact(u).cpu().numpy()
    pp = np.abs(psi) ** 2
    assert np.all(pp[got] > 0)
    _check_exact(got, psi, n, u)
    # GHZ: two non-zero amplitudes at the ends of the state
    st = sv.State(12).reset().run(C.ghz(12))
    got = st.sample_exact(rng.random(4000)).cpu().numpy()
    assert set(np.unique(got)) <= {0, (1 << 12) - 1}


@pytest.mark.parametrize("offset", [0, 1, 127])
def test_exact_one_index_per_chunk(sv, offset):
    """Non-zero probability only at index `offset` of every 128-amplitude
    chunk (the sampler's unit inside a block): each draw must land exactly
    there, the first or the last index a chunk scan reaches."""
    rng = np.random.default_rng(40 + offset)
    n = 15
    p = np.zeros(1 << n)
    p[offset::128] = rng.random((1 << n) // 128) + 0.1
    psi = np.sqrt(p / p.sum()).astype(np.complex128)
    st, psi = _upload(sv, psi)
    u = np.concatenate([[0.0, np.nextafter(1.0, 0.0)], rng.random(40000)])
    got = st.sample_exact(u).cpu().numpy()
    assert np.all(got % 128 == offset)
    _check_exact(got, psi, n, u)


def test_exact_zero_state_no_shots_and_determinism(sv):
    st = sv.State(10).from_numpy(np.zeros((1, 1 << 10), dtype=np.complex64))
    assert np.all(st.sample_exact(np.array([0.0, 0.3, 0.9])).cpu().numpy() == -1)
    st = sv.State(10).reset(37)
    assert st.sample_exact(np.zeros(0)).numel() == 0
    assert np.all(st.sample_exact(np.linspace(0, 0.999, 100)).cpu().numpy() == 37)
    rng = np.random.default_rng(3)
    st, _ = _upload(sv, pins.random_state(16, rng))
    u = rng.random(30000)
    a = st.sample_exact(u).cpu().numpy()
    b = st.sample_exact(u).cpu().numpy()
    assert np.array_equal(a, b)


def _host_z_estimate(idx, n):
    """1 - 2 c_i / S from the indices, in the same FP64 steps (integer counts)."""
    v = idx[idx >= 0]
    if v.size == 0:
        return np.full(n, np.nan)
    return np.array([1.0 - 2.0 * (float(np.count_nonzero((v >> i) & 1)) / float(v.size)) for i in range(n)])


@pytest.mark.parametrize("n,shots", [(1, 7), (5, 1000), (12, 65536 + 17), (20, 300000)])
def test_z_estimate_from_draws(sv, n, shots):
    """sv_sample_z_estimate: every <Z_i> estimate equals 1 - 2 (share of the
    draws with bit i set) computed on the host from the same indices
    (bit-equal: the counts are integers), and lies within 5 sigma of the
    oracle's exact <Z_i>."""
    rng = np.random.default_rng(n + shots)
    psi = pins.random_state(n, rng)
    st, ref = _upload(sv, psi)
    idx = st.sample_exact(rng.random(shots))
    est = st.sample_z_estimate(idx).cpu().numpy()
    want = _host_z_estimate(idx.cpu().numpy(), n)
    assert np.array_equal(est, want)
    z, norm2 = oracle.expval_z_all(ref, n)
    z = z / norm2
    sigma = np.sqrt(np.maximum(1 - z * z, 1e-12) / shots)
    assert np.all(np.abs(est - z) <= 5 * sigma + 1e-12)


def test_z_estimate_edge_cases(sv):
    st = sv.State(6).from_numpy(np.zeros((1, 1 << 6), dtype=np.complex64))
    idx = st.sample_exact(np.array([0.1, 0.5]))
    assert np.all(np.isnan(st.sample_z_estimate(idx).cpu().numpy()))       # the zero state: no index
    st = sv.State(6).reset(0b101101)
    est = st.sample_z_estimate(st.sample_exact(np.linspace(0.0, 0.99, 50))).cpu().numpy()
    assert np.array_equal(est, np.array([-1.0, 1.0, -1.0, -1.0, 1.0, -1.0]))
    assert np.all(np.isnan(st.sample_z_estimate(np.zeros(0, dtype=np.int64)).cpu().numpy()))
    L = svmod.lib()
    assert L.sv_sample_z_estimate(st.h, None, 5, None) == 1
    assert L.sv_sample_z_estimate(st.h, None, -1, None) == 1


def test_exact_bad_arguments(sv):
    st = sv.State(4).reset()
    import ctypes as C_
    L = svmod.lib()
    assert L.sv_sample_exact(st.h, 1, None, 0, None) == 1          # row out of range
    assert L.sv_sample_exact(st.h, 0, None, -1, None) == 1         # negative shots
    assert L.sv_sample_exact(st.h, 0, None, 5, None) == 1          # NULL with shots
    assert L.sv_sample_gaussian(st.h, 0, None, 10.0, None) == 1
    del C_


def test_exact_chi_square(sv):
    from scipy import stats

    rng = np.random.default_rng(12)
    n = 6
    st, psi = _upload(sv, pins.random_state(n, rng))
    p = np.abs(psi) ** 2
    p /= p.sum()
    shots = 1 << 20
    got = st.sample_exact(rng.random(shots)).cpu().numpy()
    counts = np.bincount(got, minlength=1 << n)
    chi2 = np.sum((counts - shots * p) ** 2 / (shots * p))
    assert chi2 < stats.chi2.ppf(1 - 1e-6, (1 << n) - 1)


def test_exact_full_size_properties(sv):
    """30 qubits: GHZ draws only the two ends, about half each; the first
    layer of the bench workload (a product state) gives independent bits
    with P(bit q = 1) = |U3_q[1, 0]|^2."""
    import torch

    n = 30
    rng = np.random.default_rng(30)
    shots = 1 << 20
    u = torch.as_tensor(rng.random(shots), device="cuda")
    st = sv.State(n).reset().run(C.ghz(n))
    got = st.sample_exact(u).cpu().numpy()
    assert set(np.unique(got)) <= {0, (1 << n) - 1}
    frac = np.mean(got == 0)
    assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(shots)
    full = C.brickwork_u3_cz(n, 20, 2)
    first = C.Circuit(n, list(full.ops[:n]), full.params)
    st.reset().run(first)
    got = st.sample_exact(u).cpu().numpy()
    bits = (got[:, None] >> np.arange(n)) & 1
    for q, op in enumerate(first.ops):
        col = oracle.gate_matrix("u3", [full.params[i] for i in op.params])[:, 0]
        p1 = abs(col[1]) ** 2
        assert abs(bits[:, op.targets[0]].mean() - p1) < 5 * np.sqrt(p1 * (1 - p1) / shots) + 1e-12
    st.free()


@pytest.mark.parametrize("n,seed", [(1, 1), (4, 2), (10, 3), (16, 4), (20, 5)])
def test_gaussian_parity(sv, n, seed):
    rng = np.random.default_rng(seed)
    st, psi = _upload(sv, pins.random_state(n, rng) * 0.9)
    z = rng.normal(size=1 << n)
    shots = 1e6
    y = st.sample_gaussian(z, shots).cpu().numpy()
    want = oracle.sample_gaussian(psi, n, z, shots)
    np.testing.assert_allclose(y, want, rtol=1e-9, atol=1e-9)
    assert abs(y.sum() - shots) < 1e-9 * shots


def test_gaussian_point_masses(sv):
    z = np.random.default_rng(4).normal(size=1 << 9)
    for idx in (0, 77, (1 << 9) - 1):
        st = sv.State(9).reset(idx)
        y = st.sample_gaussian(z, 1000.0).cpu().numpy()
        want = np.zeros(1 << 9)
        want[idx] = 1000.0
        np.testing.assert_allclose(y, want, atol=1e-9)


def test_gaussian_full_size(sv):
    import torch

    n = 30
    st = sv.State(n).reset().run(C.brickwork_u3_cz(n, 2, 2))
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    z = torch.randn(1 << n, dtype=torch.float64, device="cuda", generator=g)
    shots = 1e9
    y = st.sample_gaussian(z, shots)
    p = torch.view_as_real(st.tensor[0]).double().pow(2).sum(-1)
    p /= p.sum()
    assert abs(float(y.sum()) - shots) < 1e-6 * shots
    energy = float(((y - shots * p) ** 2).sum()) / shots
    expect = 1.0 - float((p * p).sum())
    assert abs(energy - expect) < 0.01
    del y, z, p
    st.free()
    torch.cuda.empty_cache()
