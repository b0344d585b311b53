import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long-running oracle check")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build()
    yield


def pytest_terminal_summary(terminalreporter):
    """Observed parity errors against their bounds, one line per check."""
    try:
        from gpu_util import RECORDS
    except ImportError:
        return
    if not RECORDS:
        return
    tr = terminalreporter
    tr.section("parity: observed error / bound")
    for test, what, obs, bound in RECORDS:
        tr.write_line(f"{obs:10.3e} / {bound:9.3e}  {test}  {what}")
