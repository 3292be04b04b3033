import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The oracle's linear algebra is on small matrices (a few hundred rows),
# where a multi-threaded BLAS spends its time synchronising its threads
# (256 x 256 eigenvalues: 0.03 s on one thread, 0.8 s on eight).
import numpy  # noqa: E402  (loads the BLAS, so that its thread count can be set)

try:
    from threadpoolctl import threadpool_limits
    _BLAS_LIMIT = threadpool_limits(limits=1, user_api="blas")
except ImportError:   # then the BLAS keeps its own thread count
    _BLAS_LIMIT = None


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")
