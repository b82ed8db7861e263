import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests that find no GPU fail loudly inside the test (the product path
    # must never fall back to the CPU); nothing is skipped silently here.
    pass


@pytest.fixture(scope="session", autouse=True)
def _built_native():
    """Build the CPU-side native pieces (generator, reference) once."""
    import netgen
    import oracle
    netgen.build(force=False)
    oracle.build(force=False)
    yield
