import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def tiny_scene():
    from paper_2307_08383_amd import scenegen
    return scenegen.tiny_scene(seed=0)


@pytest.fixture(scope="session")
def tiny_uv(tiny_scene):
    from oracle import oracle as orc
    return orc.observations(tiny_scene)


def small_scene(seed=3, n_pts=60, n_grid=3, noise=0.5, t_hi=5):
    """A scene small enough for dense linear algebra on the full Hessian."""
    from paper_2307_08383_amd import scenegen
    return scenegen.tiny_scene(seed=seed, n_pts=n_pts, n_grid=n_grid, noise_sigma=noise,
                               t_hi=t_hi, with_stats=False)
