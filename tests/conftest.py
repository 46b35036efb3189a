import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large-size case (minutes of CPU oracle time)")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def sv():
    """The HIP library binding; a GPU test fails loudly if it cannot load."""
    if not gpu_available():
        pytest.fail("GPU test selected but no GPU is visible")
    from paper_2511_19291_amd import sv as _sv
    return _sv
