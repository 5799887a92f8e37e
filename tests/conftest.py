import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(autouse=True)
def _reset_oracle_fault():
    """Every test starts with the correct oracle (mutation tests plant faults)."""
    yield
    try:
        import oracle
        if oracle._lib is not None:
            oracle.set_fault(0)
    except Exception:
        pass
