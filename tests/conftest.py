import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def load_table1():
    """Parse tests/golden/table1.txt into {case: {key: ndarray}}."""
    out, cur = {}, None
    with open(os.path.join(GOLDEN, "table1.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "case":
                cur = out.setdefault(tok[1], {})
                continue
            vals = np.array([float(t) for t in tok[1:]])
            cur[tok[0]] = vals.reshape(3, 3) if len(vals) == 9 else vals[0]
    return out


@pytest.fixture(scope="session")
def table1():
    return load_table1()


def voigt(m):
    m = np.asarray(m)
    return np.array([m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[0, 2], m[1, 2]])


def unvoigt(s):
    s = np.asarray(s)
    return np.array([[s[0], s[3], s[4]], [s[3], s[1], s[5]], [s[4], s[5], s[2]]])
