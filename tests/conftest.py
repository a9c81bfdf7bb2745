import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")

    # Under pytest-xdist every worker runs the OpenMP oracle: the cores are
    # split among the workers, since thread teams that spin at their barriers
    # slow down by orders of magnitude when they oversubscribe the machine.
    workers = os.environ.get("PYTEST_XDIST_WORKER_COUNT")
    if workers:
        import oracle

        oracle.set_threads(max(1, len(os.sched_getaffinity(0)) // int(workers)))
