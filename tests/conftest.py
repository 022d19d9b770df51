import os
import sys

# BLAS oversubscription makes the dense oracle several times slower on small
# containers; one thread per process is the fastest setting measured here.
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("OMP_NUM_THREADS", "1")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI)")
    config.addinivalue_line("markers", "slow: full-size oracle runs (minutes)")
