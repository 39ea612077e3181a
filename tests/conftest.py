import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device); parity tests proper")
    config.addinivalue_line("markers", "slow: large CPU reference runs")


@pytest.fixture(scope="session")
def orc():
    """The FP64 reference (test infrastructure), built on first use."""
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The product library on a HIP device; a missing library is an error, not a skip."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2408_06765_amd import rsi
    from paper_2408_06765_amd import _lib
    _lib.load()
    return rsi
