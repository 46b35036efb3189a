"""Workgroup order of the one-target dense sweep (sv_sweep_order_tune / _set /
_get): the order changes which workgroup moves which pairs, never the
arithmetic, so every gate's result must be bit-identical under either order;
the tuner's identity sweeps must leave the state's values unchanged; and the
default (hardware order) path stays checked against the oracle elsewhere, the
XCD-contiguous path here."""

import numpy as np
import pytest

import oracle
from paper_2511_19291_amd import circuits as C

pytestmark = pytest.mark.gpu


def test_orders_bit_identical_and_match_oracle(sv):
    n = 14
    circ = C.brickwork_u3_cz(n, 4, 41)
    st = sv.State(n)
    saved = st.sweep_order()
    try:
        outs = []
        for mask in (0, (1 << n) - 1, 0b10101010101010):
            print(f"sweep order n={n} mask={mask:#x}", flush=True)
            assert st.sweep_order(mask) == mask
            outs.append(st.reset().run(circ).to_numpy())
        for o in outs[1:]:
            assert np.array_equal(o.view(np.uint32), outs[0].view(np.uint32))
        ref = oracle.run(circ)
        assert np.max(np.abs(outs[1][0] - ref)) <= 1e-5
    finally:
        st.sweep_order(saved)
        st.free()


def test_tuner_keeps_values_and_records_choice(sv):
    n, B = 18, 2
    circ = C.brickwork_u3_cz(n, 3, 43)
    st = sv.State(n, B)
    saved = st.sweep_order()
    try:
        st.reset().run(circ)
        before = st.to_numpy()
        ms = st.tune_sweep_order()
        after = st.to_numpy()
        assert np.array_equal(before, after)             # values (a -0 may read back as +0)
        assert ms.shape == (n, 2)
        assert np.all(ms[:7] == 0) and np.all(ms[7:] > 0)
        mask = st.sweep_order()
        expect = sum(1 << t for t in range(7, n) if ms[t, 1] < ms[t, 0])
        assert mask == expect
        # gates after tuning: the same bits as in the hardware order
        a = st.reset().run(circ).to_numpy()
        st.sweep_order(0)
        b = st.reset().run(circ).to_numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    finally:
        st.sweep_order(saved)
        st.free()


def test_small_state_tunes_nothing(sv):
    st = sv.State(7)
    saved = st.sweep_order()
    ms = st.tune_sweep_order()
    assert np.all(ms == 0) and st.sweep_order() == saved
    st.free()
