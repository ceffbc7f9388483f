import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def dev():
    """The GPU device; fails loudly when the HIP extension cannot be loaded."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2104_05372_amd import dex
    dex.lib()  # raises if the library is missing
    return torch.device("cuda:0")
