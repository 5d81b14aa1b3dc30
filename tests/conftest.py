import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    O.build()
    return O


@pytest.fixture(scope="session")
def gpu():
    """A library context on cuda:0.  Fails (never skips) when the HIP library
    or the device is missing, so a GPU run cannot pass on a fallback."""
    import torch
    from paper_2208_10009_amd import sbr
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = sbr.Context(0)
    yield ctx
    ctx.close()
