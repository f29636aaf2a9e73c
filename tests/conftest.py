import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


# Summary records of parity tests (flagged-ray counts and the like): printed at
# the end of the run, and written as JSON lines to $OBBV_PARITY_JSON when set.
PARITY_RECORDS = []


def record_parity(rec):
    PARITY_RECORDS.append(dict(rec))


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    if not PARITY_RECORDS:
        return
    import json
    terminalreporter.write_sep("-", "parity records")
    for r in PARITY_RECORDS:
        terminalreporter.write_line(json.dumps(r, sort_keys=True))
    path = os.environ.get("OBBV_PARITY_JSON")
    if path:
        with open(path, "a") as f:
            for r in PARITY_RECORDS:
                f.write(json.dumps(r, sort_keys=True) + "\n")
