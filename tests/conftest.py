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


@pytest.fixture(scope="session")
def loud(pytestconfig):
    """Context manager for long host builds: the library reports its progress
    (SEAS_VERBOSE) and pytest's output capture is suspended meanwhile, so a run
    shows a line every few seconds instead of going quiet for minutes."""
    import contextlib
    capman = pytestconfig.pluginmanager.getplugin("capturemanager")

    @contextlib.contextmanager
    def cm(msg=None):
        prev = os.environ.get("SEAS_VERBOSE")
        os.environ["SEAS_VERBOSE"] = "1"
        ctx = capman.global_and_fixture_disabled() if capman is not None else contextlib.nullcontext()
        try:
            with ctx:
                if msg:
                    print(msg, flush=True)
                yield
        finally:
            if prev is None:
                os.environ.pop("SEAS_VERBOSE", None)
            else:
                os.environ["SEAS_VERBOSE"] = prev
    return cm
