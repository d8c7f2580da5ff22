"""Re-triangulation on the GPU against the oracle, point by point (needs a
GPU): the linear multi-view start and the Gauss-Newton refinement with the
cameras fixed (the alternative to Eq. (5) named in Sec. 3.1), the failure
count on a degenerate point, and the LM step that re-triangulates its
points (compared by final cost with the oracle's exact LM, which uses
Eq. (5))."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from gpu_util import T, create

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")


def _scene(kind):
    if kind == "tiny":
        return scenegen.tiny_scene(seed=0, with_stats=False)
    s = scenegen.aerial_grid_scene(seed=4, nx=10, ny=8, n_pts=20000, with_stats=False)
    if kind == "fixed":
        s.cam_fixed[[0, 9, 40, 79]] = 1
    return s


def _narrow(s, uv, cams):
    """Points whose every observation lies within normalised radius 1 (the
    radial map is increasing there, so the linear start is unique)."""
    rho = np.linalg.norm(uv, axis=0) / cams[s.obs_cam, 6]
    wide = np.zeros(s.n_pts, bool)
    np.logical_or.at(wide, s.obs_pt, rho >= 1.0)
    return ~wide


@pytest.mark.parametrize("kind", ["tiny", "mid", "fixed"])
@pytest.mark.parametrize("init,n_gn", [(True, 0), (True, 5), (False, 3)])
def test_triangulation_parity(kind, init, n_gn):
    s = _scene(kind)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    X_ref, nf_ref = P.triangulate(s.cams_init, s.pts_init, init=init, n_gn=n_gn)
    ctx = create(s, uv)
    try:
        pts = T(s.pts_init, torch.float64)
        nf = ba.ba_triangulate(ctx, T(s.cams_init, torch.float64), pts, linear_init=init, n_gn=n_gn)
        X = pts.cpu().numpy()
    finally:
        ba.ba_destroy(ctx)
    assert nf == nf_ref == 0
    err = np.abs(X - X_ref).max(axis=1) / np.maximum(1.0, np.abs(X_ref).max(axis=1))
    if init and n_gn == 0:
        sel = _narrow(s, uv, s.cams_init)
        assert sel.mean() > 0.8
        assert err[sel].max() <= 1e-9
    else:
        assert err.max() <= 1e-9


def test_triangulation_degenerate_point_counted():
    """All cameras of one point unrotated and every observation at the image
    centre: the rays coincide, the normal matrix is diag(t, t, 0) and the
    point keeps its start, as in the oracle."""
    s = scenegen.tiny_scene(seed=0, with_stats=False)
    uv = orc.project(s.cams_true, s.pts_true, s.obs_cam, s.obs_pt)
    p = 5
    ks = np.nonzero(s.obs_pt == p)[0]
    cams = s.cams_true.copy()
    cams[s.obs_cam[ks], 0:3] = 0.0
    uv[:, ks] = 0.0
    P = orc.Problem(s.n_cams, s.n_pts, s.obs_cam, s.obs_pt, uv)
    _, nf_ref = P.triangulate(cams, s.pts_init, init=True, n_gn=0, which=np.array([p], np.int32))
    ctx = create(s, uv)
    try:
        pts = T(s.pts_init, torch.float64)
        nf = ba.ba_triangulate(ctx, T(cams, torch.float64), pts, linear_init=True, n_gn=0)
        assert nf_ref == 1 and nf >= 1
        assert np.array_equal(pts.cpu().numpy()[p], s.pts_init[p])
    finally:
        ba.ba_destroy(ctx)


@pytest.mark.timeout(600)
def test_triangulation_aerial_full():
    """Every point of the 2,000-camera aerial scene (400,000 points)."""
    s = scenegen.aerial_grid_scene(seed=0, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    X_ref, nf_ref = P.triangulate(s.cams_init, s.pts_init, init=True, n_gn=4)
    ctx = create(s, uv)
    try:
        pts = T(s.pts_init, torch.float64)
        nf = ba.ba_triangulate(ctx, T(s.cams_init, torch.float64), pts, linear_init=True, n_gn=4)
        X = pts.cpu().numpy()
    finally:
        ba.ba_destroy(ctx)
    assert nf == nf_ref == 0
    err = np.abs(X - X_ref).max(axis=1) / np.maximum(1.0, np.abs(X_ref).max(axis=1))
    print(f"aerial triangulation: max rel err {err.max():.2e}")
    assert err.max() <= 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_lm_with_retriangulation(precision):
    """LM whose points are re-triangulated with the candidate cameras (3
    Gauss-Newton steps from the Eq. (5) points): its first candidate cost is
    not above the Eq. (5) candidate's, and after 15 iterations its final
    cost equals the oracle's exact LM (Eq. (5)) final cost to rel 1e-6."""
    s = _scene("mid")
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    c_ref, p_ref, _ = orc.lm_run(P, s.cams_init, s.pts_init, 15)
    F_ref = P.cost(c_ref, p_ref)
    ctx = create(s, uv, precision)
    ctx5 = create(s, uv, precision)
    try:
        cams, pts = T(s.cams_init, torch.float64), T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        hist = [ba.ba_lm_step(ctx, cams, pts, st, retriangulate=3)]
        c5, p5 = T(s.cams_init, torch.float64), T(s.pts_init, torch.float64)
        h5 = ba.ba_lm_step(ctx5, c5, p5, ba.new_lm_state(1e-4))
        assert hist[0]["accepted"] == 1 and hist[0]["tri_failed"] == 0
        assert hist[0]["cost_new"] <= h5["cost_new"] * (1 + 1e-12)
        for _ in range(14):
            hist.append(ba.ba_lm_step(ctx, cams, pts, st, retriangulate=3))
        F = P.cost(cams.cpu().numpy(), pts.cpu().numpy())
    finally:
        ba.ba_destroy(ctx)
        ba.ba_destroy(ctx5)
    print(f"LM with re-triangulation: final {F:.10e}, oracle exact LM {F_ref:.10e}")
    assert abs(F - F_ref) <= 1e-6 * F_ref
