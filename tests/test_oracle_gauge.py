"""Pins of the oracle's gauge deflation: the seven camera-space vectors are
null vectors of the undamped reduced camera system (the similarity
invariance of projection, independent of how they are computed), and the
deflated PCG reaches the dense solution with W^T r = 0 along the way."""
import numpy as np
import pytest

from oracle import fsai, gauge
from oracle import oracle as orc
from paper_2307_08383_amd import scenegen


def _problem(scene, lam):
    uv = orc.observations(scene)
    P = orc.Problem.from_scene(scene, uv)
    P.linearize(scene.cams_init, scene.pts_init)
    P.form_rcs(lam)
    blk, rhs = P.rcs()
    rp, ci = P.pattern()
    return P, fsai.dense_rcs(blk, rp, ci), rhs.ravel()


@pytest.fixture(scope="module")
def grid():
    return scenegen.aerial_grid_scene(seed=9, nx=5, ny=4, n_pts=1500, with_stats=False)


def test_gauge_vectors_are_null_vectors_of_undamped_rcs(grid):
    P, S0, _ = _problem(grid, 0.0)
    W = gauge.gauge_vectors(grid.cams_init, P.cam_row(), P.n_rows)
    # per generator, |S0 w| relative to the block scale of S0 and |w|
    for j in range(7):
        w = W[:, j]
        rel = np.linalg.norm(S0 @ w) / (np.linalg.norm(np.abs(S0) @ np.abs(w)))
        assert rel <= 1e-7, (j, rel)
    # and they are independent: W has full column rank
    sv = np.linalg.svd(W / np.linalg.norm(W, axis=0), compute_uv=False)
    assert sv[-1] > 1e-3
    # a generic vector is not in the null space (the check has teeth)
    v = np.random.default_rng(0).normal(size=W.shape[0])
    assert np.linalg.norm(S0 @ v) / np.linalg.norm(np.abs(S0) @ np.abs(v)) > 1e-3


def test_gauge_vectors_near_rotation_pi():
    # nadir cameras sit near |w| = pi; the map stays smooth there
    s = scenegen.tiny_scene(seed=1, n_pts=120, with_stats=False)
    P, S0, _ = _problem(s, 0.0)
    assert np.all(np.abs(np.linalg.norm(s.cams_init[:, :3], axis=1) - np.pi) < 0.2)
    W = gauge.gauge_vectors(s.cams_init, P.cam_row(), P.n_rows)
    for j in range(7):
        w = W[:, j]
        assert np.linalg.norm(S0 @ w) / np.linalg.norm(np.abs(S0) @ np.abs(w)) <= 1e-7


@pytest.mark.parametrize("precond", ["block_jacobi", "fsai"])
def test_deflated_pcg_solution(grid, precond):
    P, S, b = _problem(grid, 1e-6)
    W = gauge.gauge_vectors(grid.cams_init, P.cam_row(), P.n_rows)
    n = P.n_rows
    if precond == "block_jacobi":
        Minv = np.zeros_like(S)
        for i in range(n):
            Minv[9 * i:9 * i + 9, 9 * i:9 * i + 9] = np.linalg.inv(S[9 * i:9 * i + 9, 9 * i:9 * i + 9])
        M = lambda v: Minv @ v
    else:
        blk, _ = P.rcs()
        rp, ci = P.pattern()
        cnt = fsai.shared_points(n, P.cam_row(), grid.obs_cam, grid.obs_pt)
        G, _, _ = fsai.fsai(blk, rp, ci, cnt, cap=27)
        M = lambda v: G.T @ (G @ v)
    x, it, rel, worst = gauge.deflated_pcg(lambda v: S @ v, b, M, W, tol=1e-13, max_iter=3000)
    x_ref = np.linalg.solve(S, b)
    assert rel <= 1e-13
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-7 * np.abs(x_ref).max())
    # the deflation invariant W^T r_k = 0 holds along the iteration
    assert worst <= 1e-8
    # warm start: same solution
    x2, it2, rel2, _ = gauge.deflated_pcg(lambda v: S @ v, b, M, W, tol=1e-13, max_iter=3000, x_start=0.5 * x_ref)
    np.testing.assert_allclose(x2, x_ref, rtol=0, atol=1e-7 * np.abs(x_ref).max())
    # with small damping the gauge directions are the slow ones: deflation
    # needs fewer iterations than the same preconditioner alone
    _, it_plain, _ = fsai.pcg(lambda v: S @ v, b, M, tol=1e-8, max_iter=3000)
    _, it_defl, _, _ = gauge.deflated_pcg(lambda v: S @ v, b, M, W, tol=1e-8, max_iter=3000)
    assert it_defl < it_plain
