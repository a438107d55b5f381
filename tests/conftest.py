import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session", autouse=True)
def _oracle_helper():
    """The oracle's plain-C quadrature helper is compiled on demand."""
    from oracle import selfterm
    if not os.path.exists(os.path.join(ROOT, "oracle", "_selfkernel.so")):
        selfterm.build_helper()
