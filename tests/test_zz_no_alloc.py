"""The allocation-free cost entry point against ba_linearize's cost (needs
a GPU): two calls in a row on one GPU's shared buffer, the second with a
smaller input (nothing of the first may leak into it), and the size limit."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from gpu_util import T, create

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")


def _both(s):
    uv = orc.observations(s)
    cams, pts = T(s.cams_init, torch.float64), T(s.pts_init, torch.float64)
    oc, op, uvd = T(s.obs_cam, torch.int32), T(s.obs_pt, torch.int32), T(uv, torch.float64)
    cost = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    st = ba.ba_cost_noalloc(cams, pts, oc, op, uvd, cost)
    assert st == ba.BA_OK
    torch.cuda.synchronize()
    ctx = create(s, uv)
    try:
        F = ba.ba_linearize(ctx, cams, pts)
    finally:
        ba.ba_destroy(ctx)
    return float(cost.item()), F


def test_cost_noalloc_matches_linearize():
    big = scenegen.aerial_grid_scene(seed=4, nx=10, ny=8, n_pts=60000, with_stats=False)
    small = scenegen.tiny_scene(seed=1, with_stats=False)
    F1, R1 = _both(big)
    F2, R2 = _both(small)
    # both sum the same terms in different fixed orders
    assert abs(F1 - R1) <= 1e-12 * R1
    assert abs(F2 - R2) <= 1e-12 * R2
    assert small.n_obs < big.n_obs and abs(F2 - F1) > 1e-3 * F1


def test_cost_noalloc_rejects_oversize():
    s = scenegen.tiny_scene(seed=1, with_stats=False)
    uv = orc.observations(s)
    cost = torch.zeros(1, dtype=torch.float64, device="cuda")
    args = (T(s.cams_init, torch.float64), T(s.pts_init, torch.float64), T(s.obs_cam, torch.int32),
            T(s.obs_pt, torch.int32), T(uv, torch.float64), cost)
    # the size check comes before any launch: nothing is read
    assert ba.ba_cost_noalloc(*args, n_obs=134217728 + 1) == ba.BA_ERR_INVALID_ARG
    assert ba.ba_cost_noalloc(*args, n_obs=-1) == ba.BA_ERR_INVALID_ARG
    assert ba.ba_cost_noalloc(*args, n_obs=0) == ba.BA_OK
    torch.cuda.synchronize()
    assert cost.item() == 0.0
