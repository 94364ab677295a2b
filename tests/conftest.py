import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built libtt.so")
    config.addinivalue_line(
        "markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The ctypes binding, with the library loaded; skips cleanly only when
    no GPU is visible (the -m gpu tier always runs on a GPU)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1910_02371_amd import tt
    tt.lib()  # raises if libtt.so is missing
    return tt
