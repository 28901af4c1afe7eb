import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# launch shapes come from the library's defaults, not from an autotuner cache left on the machine
# (the test of the cache names its own file)
os.environ["HMC_TUNE_CACHE"] = "off"


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only oracle check")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def hip():
    """The HIP library binding; GPU tests fail loudly if it is missing."""
    if not gpu_available():
        pytest.skip("no GPU visible")
    from paper_2204_14241_amd import hmc
    return hmc
