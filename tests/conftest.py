import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Print the figures tests record with `record_property` (parity errors, ambiguous pixel
    counts), so they appear in the test report itself and not only in captured output."""
    lines = []
    for key in ("passed", "failed"):
        for rep in terminalreporter.stats.get(key, []):
            if rep.when == "call" and rep.user_properties:
                props = ", ".join(f"{k}={v}" for k, v in rep.user_properties)
                lines.append(f"{rep.nodeid} [{rep.outcome}]: {props}")
    if lines:
        terminalreporter.write_sep("-", "recorded parity figures")
        for ln in lines:
            terminalreporter.write_line(ln)
