import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# Under pytest-xdist every worker would start one OpenMP thread per core for
# the C oracles; on small grids the oversubscribed threads spin at each
# parallel region's barrier and a test of a second runs for minutes.  Share
# the cores out instead (before any OpenMP runtime starts in the worker).
if os.environ.get("PYTEST_XDIST_WORKER") and "OMP_NUM_THREADS" not in os.environ:
    _n = int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "1"))
    os.environ["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // max(1, _n)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU run of the oracle")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    O.lib()
    return O
