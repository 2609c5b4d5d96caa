import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The oracle's OpenMP sums use at most 16 threads (the GPU machine's CPU share).
os.environ.setdefault("ORACLE_THREADS", str(min(16, len(os.sched_getaffinity(0)))))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def small():
    from workloads import make_config
    return make_config(0)


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
