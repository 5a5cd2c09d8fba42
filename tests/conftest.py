import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library, loaded through the Python binding; skips without a GPU."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0911_2285_amd import ebicg

    return ebicg
