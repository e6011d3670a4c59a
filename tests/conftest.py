import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


def golden(name):
    return os.path.join(GOLDEN, name)


@pytest.fixture(scope="session")
def problems():
    from oracle.problem import Problem
    return {n: Problem.load(golden("problem_%s.json" % n)) for n in ("c1", "c2", "c3", "c4", "c5", "t1", "t2")}
