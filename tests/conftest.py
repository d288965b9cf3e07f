import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    from oracle import binding
    binding.lib()
    return binding


# Measured parity figures (GPU-oracle distances, rounding envelopes, gradient errors) that the
# tests report with record(); printed as one block at the end of the session, so that the
# figures are kept in the test log.
_RECORDS = []


def record(name, **values):
    _RECORDS.append((name, values))
    print("[parity] %s %s" % (name, " ".join("%s=%.3e" % kv if isinstance(kv[1], float)
                                               else "%s=%s" % kv for kv in values.items())),
          flush=True)


def pytest_terminal_summary(terminalreporter):
    if not _RECORDS:
        return
    terminalreporter.section("parity figures")
    for name, values in _RECORDS:
        terminalreporter.write_line("%s: %s" % (name, ", ".join(
            "%s %.3e" % kv if isinstance(kv[1], float) else "%s %s" % kv
            for kv in values.items())))


@pytest.fixture
def progress(capsys):
    """progress(msg): a line on the real terminal while a long test runs (its other output is
    captured), so that a run of several minutes is not silent."""
    def emit(msg):
        with capsys.disabled():
            print("[progress] " + msg, flush=True)
    return emit


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows
