import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large workload")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def fc():
    """The HIP binding; a GPU test that cannot load it fails loudly."""
    if not gpu_available():
        pytest.fail("gpu test collected on a machine without a GPU")
    from paper_2302_09247_amd import fastcod
    fastcod.load()
    return fastcod
