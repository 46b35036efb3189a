"""Error conventions of the C ABI on a real state:

* SV_ERR_HIP is sticky: after a HIP failure during a call on a state (forced
  from the host by the library's testing hook, so no kernel misbehaves),
  every later call on that state returns SV_ERR_HIP with the first failure's
  detail; other states are unaffected and sv_free still releases it.
* SV_ERR_CAPTURE: calls that synchronise the stream refuse to run while the
  state's stream is capturing a graph, queue nothing, and leave the state as
  it was.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

SV_ERR_HIP = 6
SV_ERR_CAPTURE = 7


def test_hip_error_is_sticky(sv):
    st = sv.State(5).reset()
    assert not st.failed
    sv.check(sv.lib().sv_inject_hip_error(st.h))
    with pytest.raises(sv.SvError) as e:
        st.reset()
    assert e.value.status == SV_ERR_HIP and "injected" in str(e.value)
    assert st.failed
    calls = [st.reset, st.expval_z_all, st.to_numpy, lambda: st.apply_gate(np.eye(2), [0]),
             lambda: st.expval([(1.0, 0, 1)])]
    for call in calls:
        with pytest.raises(sv.SvError) as e:
            call()
        assert e.value.status == SV_ERR_HIP and "earlier HIP error" in str(e.value)
    other = sv.State(5).reset()
    z = other.expval_z_all()[0]
    assert np.all(np.abs(z - 1.0) < 1e-12)
    st.free()
    other.free()


def test_synchronising_calls_refused_while_capturing(sv):
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        st = sv.State(6)
        st.reset(5)
    torch.cuda.synchronize()
    before = st.to_numpy()
    x = torch.zeros(16, device="cuda")
    g = torch.cuda.CUDAGraph()
    codes = []
    with torch.cuda.graph(g, stream=s):
        x.add_(1.0)                                   # keeps the captured graph non-empty
        for call in (st.expval_z_all, st.to_numpy, lambda: st.expval([(1.0, 0, 1)])):
            try:
                call()
                codes.append(0)
            except sv.SvError as e:
                codes.append(e.status)
    assert codes == [SV_ERR_CAPTURE] * 3
    g.replay()
    torch.cuda.synchronize()
    assert float(x[0].item()) == 1.0
    assert not st.failed
    np.testing.assert_array_equal(st.to_numpy(), before)
    z = st.expval_z_all()[0]
    assert z[0] == -1.0 and z[2] == -1.0 and z[1] == 1.0
