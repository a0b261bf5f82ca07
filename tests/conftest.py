import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def rng():
    import numpy as np
    return np.random.default_rng(12345)


@pytest.fixture(scope="session")
def config5():
    """The 1,310,720-face noisy displaced icosphere and its 16,777,216 rays,
    generated once per session (about a minute of host work)."""
    from workloads import configs as CF
    X, F = CF.mesh_config(5)
    return X, F, CF.rays_config(5, X, F)
