import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libgm.so")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def sigma_hot_table(oracle_lib):
    """The oracle's 64 x 256 table of ln(sigma_h/sigma_T), built once."""
    return oracle_lib.sigma_hot_table()
