import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU; run with -m gpu")
    config.addinivalue_line(
        "markers", "slow: CPU test that takes more than a few seconds")


def golden(name):
    """Parse a tests/golden fixture: '#' comments, then 'key v1 v2 ...'."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *vals = line.split()
            v = [float(x) for x in vals]
            out[k] = v[0] if len(v) == 1 else v
    return out


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle
