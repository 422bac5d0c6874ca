import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (gfx950) and the built HIP library")


@pytest.fixture(scope="session")
def gpu_ctx():
    """Loads the HIP library and checks that a GPU is present; fails loudly otherwise."""
    import torch
    from paper_1807_09467_amd import rsolve
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    rsolve.load()
    return torch.device("cuda:0")
