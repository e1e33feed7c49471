import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


def read_golden(name):
    """Parse a whitespace fixture under tests/golden: '#' lines are comments,
    every other line is a key followed by values."""
    path = os.path.join(ROOT, "tests", "golden", name)
    entries = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            entries.append((key, vals))
    return entries


@pytest.fixture
def golden():
    return read_golden
