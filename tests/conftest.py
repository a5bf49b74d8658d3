import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: oracle checks that take tens of seconds")


@pytest.fixture(scope="session")
def c1_mesh():
    from inputs.geometry import bar_c1
    return bar_c1()


@pytest.fixture(scope="session")
def c1_rwg(c1_mesh):
    from oracle.rwg import build_rwg
    m = c1_mesh
    return build_rwg(m.verts, m.tris, m.obj, m.n_obj)


@pytest.fixture(scope="session")
def c1_system(c1_rwg):
    """Dense FP64 oracle of the bar at 10 GHz (about 20 s on 8 cores)."""
    from oracle.operators import Physics, dense_system
    return dense_system(c1_rwg, Physics(10e9))
