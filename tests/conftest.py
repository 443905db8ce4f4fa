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
def gpu_lib():
    """The HIP library, loaded; skips cleanly only where no GPU exists."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_04671_amd import lib
    return lib.load()
