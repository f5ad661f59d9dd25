import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def pd():
    """The GPU library binding with an open context on cuda:0."""
    import torch

    import paper_2605_20816_amd as pdl
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = pdl.Context(0)
    yield pdl, ctx
    ctx.close()
