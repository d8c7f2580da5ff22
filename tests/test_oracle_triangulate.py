"""Pins of the oracle's re-triangulation (the alternative to Eq. (5) that
Sec. 3.1 names: points re-estimated from the camera poses, the cameras held
fixed), independent of how it is computed:
  - exact recovery on noise-free data, from the linear multi-view solve
    alone and after Gauss-Newton (closed form: the rays meet at the point);
  - on noisy data the result is a stationary point of each point's
    reprojection error (gradient sum Jp^T e = 0), reached from the linear
    start and from the true point alike, and equals a library least-squares
    solve (scipy) on sampled points;
  - at a converged exact-LM solution (Eq. (5) points) re-triangulation with
    the converged cameras leaves the points where they are (the LM optimum
    minimises every point's error given the cameras)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2307_08383_amd import scenegen


def _noise_free(seed=0, **kw):
    s = scenegen.tiny_scene(seed=seed, with_stats=False, **kw)
    uv = orc.project(s.cams_true, s.pts_true, s.obs_cam, s.obs_pt)
    return s, uv, orc.Problem(s.n_cams, s.n_pts, s.obs_cam, s.obs_pt, uv)


@pytest.mark.parametrize("n_gn", [0, 3])
def test_exact_recovery_noise_free(n_gn):
    s, uv, P = _noise_free()
    X, nf = P.triangulate(s.cams_true, s.pts_init, init=True, n_gn=n_gn)
    assert nf == 0
    assert np.abs(X - s.pts_true).max() <= 1e-10 * np.abs(s.pts_true).max()


def test_exact_recovery_aerial_distortion():
    """Nadir cameras with the full radial model (|k1| up to 0.05, |k2| up to
    0.01).  Where every observation of a point lies within normalised
    radius 1 the radial map r (1 + k1 r^2 + k2 r^4) is increasing and the
    linear start alone is exact; wider rays (the small grid's far cameras
    reach radius 2.3, where the map can fold back) are made exact by the
    Gauss-Newton steps."""
    s = scenegen.aerial_grid_scene(seed=5, nx=6, ny=5, n_pts=3000, with_stats=False)
    uv = orc.project(s.cams_true, s.pts_true, s.obs_cam, s.obs_pt)
    P = orc.Problem(s.n_cams, s.n_pts, s.obs_cam, s.obs_pt, uv)
    X, nf = P.triangulate(s.cams_true, np.zeros_like(s.pts_true), init=True, n_gn=0)
    assert nf == 0
    rho = np.linalg.norm(uv, axis=0) / s.cams_true[s.obs_cam, 6]
    wide = np.zeros(s.n_pts, bool)
    np.logical_or.at(wide, s.obs_pt, rho >= 1.0)
    assert (~wide).sum() > 0.9 * s.n_pts
    assert np.abs(X[~wide] - s.pts_true[~wide]).max() <= 1e-9
    X, nf = P.triangulate(s.cams_true, np.zeros_like(s.pts_true), init=True, n_gn=4)
    assert nf == 0
    assert np.abs(X - s.pts_true).max() <= 1e-9


def _point_gradients(s, uv, cams, X):
    F, e, Jc, Jp = orc.linearize(cams, X, s.obs_cam, s.obs_pt, uv)
    g = np.zeros((s.n_pts, 3))
    a = np.zeros(s.n_pts)
    np.add.at(g, s.obs_pt, np.einsum("krj,kr->kj", Jp, e))
    np.add.at(a, s.obs_pt, np.linalg.norm(Jp.reshape(-1, 6), axis=1) * np.linalg.norm(e, axis=1))
    return F, g, a


def test_noisy_stationary_and_start_independent():
    s = scenegen.tiny_scene(seed=1, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    X_lin, nf = P.triangulate(s.cams_init, s.pts_init, init=True, n_gn=8)
    assert nf == 0
    X_true_start, nf2 = P.triangulate(s.cams_init, s.pts_true, init=False, n_gn=8)
    assert nf2 == 0
    assert np.abs(X_lin - X_true_start).max() <= 1e-10 * np.abs(X_lin).max()
    F, g, a = _point_gradients(s, uv, s.cams_init, X_lin)
    assert (np.linalg.norm(g, axis=1) / a).max() <= 1e-9
    # no other point position does better: the cost is not above the start's
    F0 = orc.linearize(s.cams_init, s.pts_init, s.obs_cam, s.obs_pt, uv)[0]
    assert F <= F0


def test_matches_library_least_squares():
    from scipy.optimize import least_squares
    s = scenegen.aerial_grid_scene(seed=6, nx=5, ny=4, n_pts=400, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    X, nf = P.triangulate(s.cams_init, s.pts_init, init=True, n_gn=8)
    assert nf == 0
    for p in range(0, s.n_pts, 37):
        ks = np.nonzero(s.obs_pt == p)[0]

        def resid(x):
            pred = orc.project(s.cams_init, x.reshape(1, 3), s.obs_cam[ks], np.zeros(len(ks), np.int32))
            return (pred - uv[:, ks]).ravel()
        sol = least_squares(resid, s.pts_init[p], jac="3-point", xtol=1e-15, ftol=1e-15, gtol=1e-15)
        # the library's finite-difference Jacobian limits it to ~1e-8; the
        # oracle's point must be at least as good and agree to that level
        assert np.abs(sol.x - X[p]).max() <= 1e-6 * max(1.0, np.abs(X[p]).max()), p
        assert np.sum(resid(X[p]) ** 2) <= np.sum(sol.fun ** 2) * (1 + 1e-12), p


def test_leaves_converged_lm_points_in_place():
    s = scenegen.tiny_scene(seed=2, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    cams, pts, hist = orc.lm_run(P, s.cams_init, s.pts_init, 40, tol=1e-12, max_iter=5000)
    X, nf = P.triangulate(cams, pts, init=False, n_gn=5)
    assert nf == 0
    F_lm = P.cost(cams, pts)
    F_tri = P.cost(cams, X)
    assert F_tri <= F_lm * (1 + 1e-12) and F_lm - F_tri <= 1e-9 * F_lm
    assert np.abs(X - pts).max() <= 1e-6 * np.abs(pts).max()
    # from the linear start as well
    X2, _ = P.triangulate(cams, pts, init=True, n_gn=8)
    assert np.abs(X2 - pts).max() <= 1e-6 * np.abs(pts).max()


def test_subset_and_degenerate_point():
    """Only the listed points change; a point whose rays are all parallel
    has a singular normal matrix and keeps its start."""
    s, uv, P = _noise_free()
    which = np.array([3, 10, 42], np.int32)
    start = s.pts_init.copy()
    X, nf = P.triangulate(s.cams_true, start, init=True, n_gn=2, which=which)
    assert nf == 0
    keep = np.ones(s.n_pts, bool)
    keep[which] = False
    assert np.array_equal(X[keep], start[keep])
    assert np.abs(X[which] - s.pts_true[which]).max() <= 1e-10
    # every camera of point p unrotated (R = I exactly) and every
    # observation at the image centre: all rays are the optical axis
    # direction, so the normal matrix is diag(t, t, 0) exactly
    p = 5
    ks = np.nonzero(s.obs_pt == p)[0]
    cams = s.cams_true.copy()
    cams[s.obs_cam[ks], 0:3] = 0.0
    uv2 = uv.copy()
    uv2[:, ks] = 0.0
    P2 = orc.Problem(s.n_cams, s.n_pts, s.obs_cam, s.obs_pt, uv2)
    X, nf = P2.triangulate(cams, start, init=True, n_gn=0, which=np.array([p], np.int32))
    assert nf == 1 and np.array_equal(X[p], start[p])
