"""Gauge-deflated PCG on the GPU against the oracle (needs a GPU): the gauge
vectors, deflated solves with block-Jacobi and FSAI preconditioners (also
with fixed cameras), and LM runs with deflation."""
import numpy as np
import pytest

from oracle import fsai, gauge
from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from gpu_util import T, create

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")


def _case(scene, lam, cam_fixed=None):
    uv = orc.observations(scene)
    P = orc.Problem(scene.n_cams, scene.n_pts, scene.obs_cam, scene.obs_pt, uv, cam_fixed)
    P.linearize(scene.cams_init, scene.pts_init)
    P.form_rcs(lam)
    ctx = create(scene, uv, 0, cam_fixed=cam_fixed)
    ba.ba_linearize(ctx, T(scene.cams_init, torch.float64), T(scene.pts_init, torch.float64))
    ba.ba_form_rcs(ctx, lam)
    return P, ctx


def _scene():
    return scenegen.aerial_grid_scene(seed=4, nx=10, ny=8, n_pts=12000, with_stats=False)


def test_gauge_vectors_parity():
    s = _scene()
    P, ctx = _case(s, 1e-4)
    try:
        Wg = ba.ba_get_gauge(ctx)
    finally:
        ba.ba_destroy(ctx)
    W = gauge.gauge_vectors(s.cams_init, P.cam_row(), P.n_rows)
    Wg = Wg.transpose(0, 2, 1).reshape(-1, 7)      # [row][vec][comp] -> [row*9+comp][vec]
    for j in range(7):
        ref = W[:, j]
        assert np.linalg.norm(Wg[:, j] - ref) <= 1e-7 * np.linalg.norm(ref), j


@pytest.mark.parametrize("precond", ["block_jacobi", "fsai"])
@pytest.mark.parametrize("fixed", [False, True])
def test_deflated_pcg_parity(precond, fixed):
    s = _scene()
    cf = None
    if fixed:
        cf = np.zeros(s.n_cams, np.uint8)
        cf[[0, 1, 37]] = 1
    lam = 1e-7
    P, ctx = _case(s, lam, cf)
    pre = ba.BA_PRECOND_FSAI if precond == "fsai" else ba.BA_PRECOND_BLOCK_JACOBI
    try:
        dxc = torch.empty((P.n_rows, 9), dtype=torch.float64, device="cuda")
        info = ba.ba_pcg_solve(ctx, dxc, tol=1e-12, max_iter=6000, precond=pre, deflate=True)
        x = dxc.cpu().numpy().ravel()
        i6 = ba.ba_pcg_solve(ctx, dxc, tol=1e-6, max_iter=3000, precond=pre, deflate=True)
        x6 = dxc.cpu().numpy().ravel()
        p6 = ba.ba_pcg_solve(ctx, dxc, tol=1e-6, max_iter=3000, precond=pre)
        # warm start
        ba.ba_pcg_solve(ctx, dxc, tol=1e-3, precond=pre, deflate=True)
        w = ba.ba_pcg_solve(ctx, dxc, tol=1e-10, max_iter=6000, precond=pre, deflate=True, x0=dxc.clone())
        xw = dxc.cpu().numpy().ravel()
    finally:
        ba.ba_destroy(ctx)
    blk, rhs = P.rcs()
    rp, ci = P.pattern()
    S = fsai.dense_rcs(blk, rp, ci)
    b = rhs.ravel()
    x_ref = np.linalg.solve(S, b)
    assert info["status"] == 0 and info["relres"] <= 1e-12
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-6 * np.abs(x_ref).max())
    assert w["status"] == 0
    np.testing.assert_allclose(xw, x_ref, rtol=0, atol=1e-4 * np.abs(x_ref).max())
    if precond == "fsai":
        cnt = fsai.shared_points(P.n_rows, P.cam_row(), s.obs_cam, s.obs_pt)
        G, _, _ = fsai.fsai(blk, rp, ci, cnt, cap=27)
        M = lambda v: G.T @ (G @ v)
    else:
        Minv = np.zeros_like(S)
        for i in range(P.n_rows):
            Minv[9 * i:9 * i + 9, 9 * i:9 * i + 9] = np.linalg.inv(S[9 * i:9 * i + 9, 9 * i:9 * i + 9])
        M = lambda v: Minv @ v
    W = gauge.gauge_vectors(s.cams_init, P.cam_row(), P.n_rows)
    _, it_ref, _, _ = gauge.deflated_pcg(lambda v: S @ v, b, M, W, tol=1e-6, max_iter=3000)
    assert i6["status"] == 0 and abs(i6["iters"] - it_ref) <= max(3, 0.1 * it_ref)
    assert np.linalg.norm(b - S @ x6) <= 1.5e-6 * np.linalg.norm(b)
    # deflation never costs iterations beyond rounding (here, with fixed
    # cameras anchoring the gauge, the seven directions are slow modes and
    # removing them saves iterations)
    assert i6["iters"] <= p6["iters"] + 3
    if fixed:
        assert i6["iters"] < 0.8 * p6["iters"]


@pytest.mark.parametrize("precond", ["block_jacobi", "fsai"])
def test_lm_with_deflation_final_cost(precond):
    s = scenegen.aerial_grid_scene(seed=7, nx=8, ny=6, n_pts=6000, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    c_ref, p_ref, _ = orc.lm_run(P, s.cams_init, s.pts_init, 12)
    F_ref = P.cost(c_ref, p_ref)
    pre = ba.BA_PRECOND_FSAI if precond == "fsai" else ba.BA_PRECOND_BLOCK_JACOBI
    ctx = create(s, uv, 1)
    try:
        cams = T(s.cams_init, torch.float64)
        pts = T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        for _ in range(12):
            info = ba.ba_lm_step(ctx, cams, pts, st, precond=pre, deflate=True)
            assert info["pcg_status"] in (0, ba.BA_ERR_NOT_CONVERGED)
        F = P.cost(cams.cpu().numpy(), pts.cpu().numpy())
    finally:
        ba.ba_destroy(ctx)
    assert abs(F - F_ref) <= 1e-6 * F_ref
