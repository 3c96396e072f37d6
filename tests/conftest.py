import os
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the autotuner's persistent cache goes to a per-session temporary file, not
# the user's cache directory (set before the library's first table lookup)
os.environ.setdefault("QSVM_TUNE_CACHE", os.path.join(tempfile.gettempdir(), f"qsvm_tune_tests_{os.getpid()}.txt"))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")
