import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take tens of seconds")


_GRIDS = {}


@pytest.fixture(scope="session")
def oracle_grid():
    """Cached oracle grids by level (building J=5 takes ~0.1 s, J=6 ~0.5 s)."""
    from oracle.grid import Grid

    def get(J):
        if J not in _GRIDS:
            _GRIDS[J] = Grid(J)
        return _GRIDS[J]
    return get
