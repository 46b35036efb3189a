"""The allocation-free <Z_i> entry point (sv_expval_z_all_noalloc) against
sv_expval_z_all, the entry point whose kernels it shares.

Both run the same two kernels with the same fixed summation order, so their
outputs must agree bit for bit; the values are also checked against the
oracle's <Z_i> of the same complex64 amplitudes. Two calls in a row on one
GPU, the second on a smaller state, exercise the shared fixed buffer (it keeps
the first call's partials; the second must not read them). The largest shape
the buffer admits runs too, and one shape beyond it is refused before
anything is queued.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2511_19291_amd import circuits as C

pytestmark = pytest.mark.gpu

SV_ERR_UNSUPPORTED = 4


def _noalloc(st):
    out = torch.full((st.batch, st.n + 1), float("nan"), dtype=torch.float64, device=st.tensor.device)
    st.expval_z_all_into(out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _prepared(sv, n, batch, seed):
    circ = C.hea_ladder(n, 2, seed)
    rng = np.random.default_rng(seed)
    params = rng.uniform(0, 2 * np.pi, size=(batch, circ.n_params))
    st = sv.State(n, batch).reset()
    st.run(circ, params)
    return st


@pytest.mark.parametrize("first,second", [((20, 3), (12, 2)), ((16, 1), (9, 5)), ((14, 4), (3, 1))])
def test_noalloc_matches_allocating_entry_point(sv, first, second):
    for (n, batch), seed in ((first, 101), (second, 102)):
        print(f"noalloc case n={n} batch={batch} seed={seed}", flush=True)
        st = _prepared(sv, n, batch, seed)
        got = _noalloc(st)
        ref = st.expval_z_all()
        assert np.array_equal(got, ref), np.max(np.abs(got - ref))
        psi = st.to_numpy()
        for r in range(batch):
            z, norm2 = oracle.expval_z_all(psi[r].astype(np.complex128), n)
            assert np.max(np.abs(got[r, :n] - z)) <= 1e-12
            assert abs(got[r, n] - norm2) <= 1e-12
        st.free()


def test_noalloc_largest_shape_then_smaller(sv):
    # n = 28 at batch 4 needs 4 * 2^14 * 15 = 983 040 of the 1 048 576 partials
    print("noalloc case n=28 batch=4", flush=True)
    st = sv.State(28, 4).reset(0)
    st.apply_gate(np.array([[1, 1], [1, -1]]) / np.sqrt(2), [27])
    st.apply_gate(np.array([[np.cos(0.3), -np.sin(0.3)], [np.sin(0.3), np.cos(0.3)]]), [5])
    got = _noalloc(st)
    ref = st.expval_z_all()
    assert np.array_equal(got, ref)
    expect = np.ones(29)
    expect[27] = 0.0
    expect[5] = np.cos(0.6)
    assert np.max(np.abs(got[:, :28] - expect[:28])) <= 1e-6
    assert np.max(np.abs(got[:, 28] - 1.0)) <= 1e-6
    st.free()
    print("noalloc case n=10 batch=2 after the largest", flush=True)
    small = _prepared(sv, 10, 2, 103)
    got = _noalloc(small)
    assert np.array_equal(got, small.expval_z_all())
    small.free()


def test_noalloc_refuses_beyond_buffer(sv):
    # n = 28 at batch 5 would need 1 228 800 partials: refused before any launch
    print("noalloc case n=28 batch=5 (refused)", flush=True)
    st = sv.State(28, 5)
    out = torch.zeros((5, 29), dtype=torch.float64, device="cuda")
    with pytest.raises(sv.SvError) as e:
        st.expval_z_all_into(out)
    assert e.value.status == SV_ERR_UNSUPPORTED and "fixed buffer" in str(e.value)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    st.free()
