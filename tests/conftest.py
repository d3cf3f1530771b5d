import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU statistics tests")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Compile the CPU oracle once per session if it is missing or stale."""
    from oracle import build as ob
    src = os.path.join(ROOT, "oracle", "smc_oracle.c")
    lib = ob.LIB
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        ob.build()
    yield
