import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libpiv.so")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """One line with every parity exemption granted in the session (near-tie
    peaks, near-flat windows, near-threshold validation decisions and their
    propagation), so that the counts appear in the run's output."""
    try:
        import _helpers
    except ImportError:
        return
    ex = getattr(_helpers, "EXEMPTIONS", [])
    tot = {}
    for _, kind, n in ex:
        tot[kind] = tot.get(kind, 0) + n
    body = ", ".join(f"{k} {v}" for k, v in sorted(tot.items())) or "none"
    terminalreporter.write_line(f"parity exemptions: {body}")
    for where, kind, n in ex:
        terminalreporter.write_line(f"  {where}: {kind} {n}")
