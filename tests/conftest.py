import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on cuda:0.  A GPU test fails (does not skip) when no
    device is visible: a silent skip would hide a missing GPU path."""
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    import paper_1203_1692_amd as sp
    sp.load()
    return sp
