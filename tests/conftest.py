import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


# The host-sanitizer test runs the CPU tests of the library against a
# sanitizer build of it: HK_TEST_LIB names that build.
if os.environ.get("HK_TEST_LIB"):
    from paper_1405_1931_amd import _lib as _hk_lib

    _hk_lib.LIB_PATH = os.environ["HK_TEST_LIB"]


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size workload (minutes on the CPU side)")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    return oracle.load()
