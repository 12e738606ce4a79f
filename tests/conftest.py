import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def load_paper_constants():
    """Parse tests/golden/d2q9_paper.txt (values typed from the paper)."""
    from fractions import Fraction

    import numpy as np

    vel, w, M, relaxed = None, None, [], None
    with open(os.path.join(GOLDEN, "d2q9_paper.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            if key == "velocities":
                vel = np.array([[int(c) for c in v.split(",")] for v in vals], dtype=np.int64)
            elif key == "weights":
                w = np.array([float(Fraction(v)) for v in vals])
            elif key == "M":
                M.append([int(v) for v in vals])
            elif key == "relaxed":
                relaxed = [int(v) for v in vals]
    return vel, w, np.array(M, dtype=np.float64), relaxed


@pytest.fixture(scope="session")
def paper_constants():
    return load_paper_constants()
