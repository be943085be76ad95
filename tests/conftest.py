import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP path, loaded through its C ABI; skips only when no GPU exists."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_08679_amd import ebe
    ebe.load()  # raises loudly if the library is missing
    return ebe
