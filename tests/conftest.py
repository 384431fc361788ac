import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build()
    yield


def pytest_terminal_summary(terminalreporter):
    """Largest measured error per (quantity, precision) of the GPU parity
    tests against the oracle, and the test that produced it."""
    try:
        from tests.gpu_util import MEASURED
    except Exception:
        return
    if not MEASURED:
        return
    worst = {}
    for test, what, prec, v in MEASURED:
        k = (what, prec)
        if k not in worst or v > worst[k][0]:
            worst[k] = (v, test)
    terminalreporter.write_line("measured errors against the oracle (largest per quantity and precision):")
    for (what, prec), (v, test) in sorted(worst.items()):
        terminalreporter.write_line(f"  {what:8s} {prec:10s} {v:.3e}  {test}")
