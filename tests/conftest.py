import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session", autouse=True)
def built_library():
    """The in-tree HIP library, compiled here (hipcc cross-compiles for gfx950 without a
    GPU) when a clean checkout has none; the host-side tests load it on the CPU."""
    from paper_2607_13740_amd import build as B
    from paper_2607_13740_amd import gracedg as G
    if not os.path.exists(G.LIB_PATH):
        B.build()
    return G.LIB_PATH


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O.build(force=False)
    return O
