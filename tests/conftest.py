import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def tiny_mesh_factory():
    """Small quadtree meshes with hanging nodes and five levels (16x16 base
    cells reached from a 4x4 coarse grid, two local refinements in the band
    |x| < 3, |y| < 1)."""
    from oracle.mesh import Mesh
    cache = {}

    def make(p):
        if p not in cache:
            cache[p] = Mesh(16, 2, p, coarse=4, band=(3.0, 1.0))
        return cache[p]
    return make
