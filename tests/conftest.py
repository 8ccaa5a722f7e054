import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Compile the CPU oracle if it has not been built yet (gcc, seconds)."""
    from oracle import build as obuild

    if not os.path.exists(os.path.join(ROOT, "oracle", "liboo_oracle.so")):
        obuild.build()
    yield
