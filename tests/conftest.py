import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as o
    o.lib()
    return o


@pytest.fixture(scope="session")
def wl():
    from paper_1503_01725_amd import workloads
    return workloads


@pytest.fixture(scope="session")
def N():
    from paper_1503_01725_amd import _native
    _native.lib()
    return _native


@pytest.fixture(scope="session")
def eng():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1503_01725_amd import engine
    return engine
