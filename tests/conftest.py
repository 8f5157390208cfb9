import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (gfx950)")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.path.exists(oracle.SO):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def qtn():
    so = os.path.join(ROOT, "paper_2204_06045_amd", "libqtn.so")
    if not os.path.exists(so):
        from paper_2204_06045_amd import build
        build.build()
    import paper_2204_06045_amd as Q
    return Q


@pytest.fixture(scope="session")
def gpu(qtn):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no HIP device is visible")
    return torch.device("cuda:0")
