import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def pw():
    """The HIP library's Python face; GPU tests fail (not skip) without a GPU."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU (run with -m 'not gpu' on a CPU host)")
    import paper_2507_08578_amd as pwmod
    return pwmod


@pytest.fixture(scope="session")
def ctx(pw):
    return pw.Context(0)
