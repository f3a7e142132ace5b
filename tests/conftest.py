import os
import sys

for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

try:  # small dense operations dominate the oracle; threaded BLAS only slows them down
    import threadpoolctl
    _LIMITS = threadpoolctl.threadpool_limits(1)
except Exception:  # pragma: no cover
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI)")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
