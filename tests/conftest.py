import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    """Build the two host-only libraries (generators, FP64 reference) if absent."""
    from paper_1901_06229_amd import synth
    import oracle
    if not os.path.exists(synth.LIB_PATH):
        synth.build()
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    yield
