import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def tmpdata(tmp_path_factory):
    """A private tmpfs-backed data directory for files a test creates."""
    base = "/dev/shm" if os.path.isdir("/dev/shm") else None
    import tempfile
    d = tempfile.mkdtemp(prefix="gsys_test_", dir=base)
    yield d
    import shutil
    shutil.rmtree(d, ignore_errors=True)
