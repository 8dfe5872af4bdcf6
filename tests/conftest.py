import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a gfx950 GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionfinish(session, exitstatus):
    """Write the values the parity tests measured (tests/parity.py) where CTFISS_PARITY_LOG says."""
    path = os.environ.get("CTFISS_PARITY_LOG")
    if not path:
        return
    import json

    try:
        from parity import RECORDS
    except ImportError:
        return
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    with open(path, "w") as f:
        json.dump(RECORDS, f, indent=1)
