import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle
    return oracle


@pytest.fixture(scope="session")
def msm():
    """The ctypes binding; importing it fails loudly if libmsm.so is missing."""
    from paper_0904_3151_amd import msm as M
    return M


@pytest.fixture(scope="session")
def ctx(msm):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = msm.Context(0)
    yield c
    c.close()


def announce(*parts):
    """Print and flush the case name before a GPU step."""
    print("[gpu-case]", *parts, flush=True)
