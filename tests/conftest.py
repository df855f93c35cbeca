import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _native_inputs():
    """Build the CPU-side helper libraries (oracle, test function) if absent."""
    import oracle
    import workloads.synth as ws
    oracle.build_library(force=False)
    ws.build_testfn(force=False)
    yield


def golden(name):
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows
