import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built libkotssn.so")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def gpu_ctx():
    """A library context on cuda:0.  Fails (not skips) when the GPU or the library is missing."""
    import torch
    from paper_2310_14087_amd import kotssn
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    ctx = kotssn.Context(0)
    yield ctx
    ctx.close()
