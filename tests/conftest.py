import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libpphd.so")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The binding, with the library loaded and a GPU present (fails loudly otherwise)."""
    import torch
    from paper_1503_03769_amd import pphd
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    pphd.lib()
    return pphd
