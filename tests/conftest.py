import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU statistics")


GOLDEN = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="session")
def orc():
    from oracle import coracle
    coracle.build(force=False)
    return coracle


@pytest.fixture(scope="session")
def zg():
    """The HIP library through its Python binding (GPU tests only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_19493_amd as Z
    return Z


@pytest.fixture(scope="session")
def ctx(zg):
    c = zg.Context(0)
    yield c
    c.close()
