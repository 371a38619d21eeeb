import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def hiplib():
    """The built HIP library (built here on first use if it is missing)."""
    from paper_2411_05771_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    return b.LIB


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def skei(hiplib):
    if not gpu_available():
        pytest.fail("GPU tests need a HIP device (run them with -m gpu on an MI355X)")
    from paper_2411_05771_amd import ops
    return ops
