import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: longer CPU runs of the oracle")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def W():
    from paper_2112_08035_amd import workloads
    return workloads


@pytest.fixture(scope="module")
def S():
    """The library binding on a GPU machine; GPU tests skip without a device.
    (Host-side test modules define their own S that needs no device.)"""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_08035_amd import smcrt
    smcrt.lib()
    return smcrt


@pytest.fixture(scope="module")
def eng(S):
    e = S.Engine(0)
    yield e
    e.close()
