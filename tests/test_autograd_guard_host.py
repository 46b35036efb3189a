"""Host logic of the autograd layers' stale-state guard (no GPU): the
version recorded at forward must equal the state's version at backward, and
the drift of the recomputed start state must stay within DRIFT_MAX."""

import types

import numpy as np
import pytest

from paper_2511_19291_amd import autograd as AG


def test_version_guard():
    state = types.SimpleNamespace(version=3)
    ctx = types.SimpleNamespace()
    AG._saved_version(ctx, state)
    AG._check_fresh(ctx)              # unchanged: accepted
    state.version += 1
    with pytest.raises(AG.StaleStateError):
        AG._check_fresh(ctx)


def test_drift_guard():
    AG._check_drift(np.array([0.0, 1e-6, AG.DRIFT_MAX]))
    AG._check_drift(np.zeros(0))
    with pytest.raises(AG.StaleStateError):
        AG._check_drift(np.array([1e-7, 2 * AG.DRIFT_MAX]))
    with pytest.raises(AG.StaleStateError):
        AG._check_drift(np.array([np.nan]))
