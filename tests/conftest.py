import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU case")


@pytest.fixture(scope="session", autouse=True)
def _private_tune_cache(tmp_path_factory):
    """Tests that autotune record their winners in a cache of their own, never
    in a cache the caller's environment names."""
    old = os.environ.get("HJ_TUNE_CACHE")
    os.environ["HJ_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "cache.txt")
    yield
    if old is None:
        os.environ.pop("HJ_TUNE_CACHE", None)
    else:
        os.environ["HJ_TUNE_CACHE"] = old


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    # The generator and the oracle are plain gcc builds; compile them when absent.
    from paper_2002_12115_amd import inputs
    import oracle
    inputs.build()
    oracle.build()
    yield
