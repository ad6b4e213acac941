import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


def pytest_terminal_summary(terminalreporter):
    from parity_log import RECORDS

    if not RECORDS:
        return
    terminalreporter.write_sep("-", "measured parity errors (largest per test, against its bar)")
    for name, err, bar in RECORDS:
        terminalreporter.write_line(f"[parity] {name}: {err:.3e} (bar {bar:.0e})")
