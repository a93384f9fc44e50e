import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def hsvd_ctx():
    """A library context on cuda:0 (GPU tests only)."""
    import torch

    from paper_1008_1371_amd import hsvd as H
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = H.Context(0)
    yield ctx
    ctx.close()
