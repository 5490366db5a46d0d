import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU case")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built C-ABI library, loaded once.  GPU tests fail loudly when it is missing."""
    import torch
    from paper_1711_03789_amd import mx
    assert torch.cuda.is_available(), "gpu tests need a GPU"
    mx.load()
    return mx
