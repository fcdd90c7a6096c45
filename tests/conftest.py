import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.dirname(os.path.abspath(__file__))
for _p in (ROOT, TESTS):
    if _p not in sys.path:
        sys.path.insert(0, _p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=not os.path.exists(oracle.LIB_PATH))
    return oracle


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    import parity_log
    if parity_log.LINES:
        terminalreporter.section("parity against the oracle")
        for line in parity_log.LINES:
            terminalreporter.write_line(line)
