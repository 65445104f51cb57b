import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long-running (full-size configurations)")


@pytest.fixture(scope="session")
def oracle_bin():
    import oracle
    return oracle.build(force=False)


@pytest.fixture(scope="session")
def cflr_lib():
    """The built library (no device needed to load it)."""
    import paper_2401_11029_amd as cflr
    return cflr.lib()


@pytest.fixture(scope="session")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test on a machine without a HIP device"
    import paper_2401_11029_amd as cflr
    c = cflr.Context(0)
    yield c
    c.close()
