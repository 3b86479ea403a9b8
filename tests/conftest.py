import os
import sys

import pytest

# parallel test workers each load the OpenMP oracle: keep their threads few so
# the workers do not oversubscribe the cores (read when the oracle loads)
if "PYTEST_XDIST_WORKER" in os.environ:
    os.environ.setdefault("OMP_NUM_THREADS", "2")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that runs for more than ~10 s")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    return oracle
