import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running (full-size workload)")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def rb():
    """The product binding; on a machine with a GPU its HIP library must load."""
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_1805_06124_amd as rbmod
    rbmod.load()  # raises if the HIP library is missing
    return rbmod
