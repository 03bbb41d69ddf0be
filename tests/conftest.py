import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle

    return oracle.get()


@pytest.fixture(scope="session")
def gctx():
    """One library context on cuda:0 for the GPU tests."""
    import torch

    from paper_2107_13887_amd import rbfdef

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    h = rbfdef.rbf_ctx_create(0)
    yield h
    torch.cuda.synchronize()
    rbfdef.rbf_ctx_destroy(h)

