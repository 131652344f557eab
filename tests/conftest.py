import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def ff():
    from pe_melt import polyethylene_forcefield
    return polyethylene_forcefield()


@pytest.fixture(scope="session")
def melt3k():
    """The 3,000-atom melt (10 chains, 0.80 g/cm^3, 500 K) with 0.05 A jitter."""
    from pe_melt import make_melt
    return make_melt(10, density=0.80, T=500.0, seed_melt=1000, seed_vel=1001, jitter=0.05)


def golden(name):
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows[key] = np.array([int(v) for v in vals])
    return rows
