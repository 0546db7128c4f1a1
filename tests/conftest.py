import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU run (closed-form steady states)")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def torch_stream():
    """torch's current stream on cuda:0, handed to the library."""
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch.cuda.current_stream().cuda_stream
