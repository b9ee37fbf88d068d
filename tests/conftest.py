import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding (fails loudly if missing)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_01265_amd as sts
    sts.load()
    return sts
