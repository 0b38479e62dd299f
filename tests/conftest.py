import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C ABI)")
    config.addinivalue_line("markers", "slow: long CPU-side check")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session", autouse=True)
def _private_tune_cache(tmp_path_factory):
    """Batches the tests autotune store their shapes in a file of this test
    session, not in the user's cache directory."""
    if "RT_TUNE_CACHE" not in os.environ:
        os.environ["RT_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "tune.json")
    yield
