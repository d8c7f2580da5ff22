"""Shared intrinsics on the GPU against the reference (needs a GPU): images
with 6 exterior unknowns taking the 5 interior unknowns of their physical
camera (Sec. 4.1's c = 11; Table 2's fewer cameras than images).

  - the block pattern over image and camera rows, bit-exact;
  - the RCS as padded 9x9 blocks (identity on the unused diagonal slots,
    zero elsewhere) and its right-hand side against the reference's
    point-by-point elimination: per-block error 1e-10 (FP64, floored metric)
    and rhs 1e-9; with one and several physical cameras and fixed images;
  - PCG on it against the dense solution, its unused slots exactly 0;
  - LM: the step (PCG to rel 1e-12) against the reference's dense step of
    Eq. (1), and the trajectory of 8 iterations against the reference's LM
    (same damping schedule), final cost to rel 1e-6;
  - the same with points seen by more than 64 images (tracks longer than a
    wave, which the fused stage and back-substitution take one workgroup
    per point), up to every image of a 272-image block."""
import numpy as np
import pytest

from oracle import intrinsics as I
from paper_2307_08383_amd import scenegen

from gpu_util import T, block_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")


def _case(kind):
    if kind == "small":
        s = scenegen.shared_intrinsics_scene(seed=5, nx=4, ny=3, n_pts=300, n_phys=3)
    elif kind == "one_camera":
        s = scenegen.shared_intrinsics_scene(seed=6, nx=5, ny=4, n_pts=600, n_phys=1)
    elif kind == "fixed":
        s = scenegen.shared_intrinsics_scene(seed=7, nx=5, ny=4, n_pts=600, n_phys=3)
        s.img_fixed[[0, 7, 19]] = 1
    elif kind == "long":
        # points seen by 65 .. all 272 images (more than a 64-wide wave, up
        # to two passes of a 256-thread workgroup), three images fixed
        s = scenegen.shared_intrinsics_scene(seed=9, nx=17, ny=16, n_pts=800, n_phys=3,
                                             long_tracks=(65, 100, 200, 256, 257, 272))
        s.img_fixed[[0, 100, 271]] = 1
    elif kind == "long_small":
        s = scenegen.shared_intrinsics_scene(seed=10, nx=10, ny=8, n_pts=400, n_phys=2, long_tracks=(65, 72, 80))
    else:   # mid: 80 images, 4 cameras, several tiles of every kernel
        s = scenegen.shared_intrinsics_scene(seed=8, nx=10, ny=8, n_pts=4000, n_phys=4)
    pu, pv = I.project(s.ext_true, s.intr_true, s.img_cam, s.pts_true, s.obs_img, s.obs_pt)
    uv = np.stack([pu.v, pv.v]) + s.noise
    P = I.SharedProblem(s.n_img, s.n_phys, s.img_cam, s.n_pts, s.obs_img, s.obs_pt, uv, s.img_fixed)
    return s, uv, P


def _ctx(s, uv):
    return ba.ba_create_shared(s.n_img, s.n_phys, s.n_pts, T(s.obs_img, torch.int32), T(s.obs_pt, torch.int32),
                               T(uv, torch.float64), T(s.img_cam, torch.int32),
                               T(s.img_fixed, torch.uint8) if s.img_fixed.any() else None)


def _params(ext, intr):
    return T(np.concatenate([ext.ravel(), intr.ravel()]), torch.float64)


@pytest.mark.parametrize("kind", ["small", "one_camera", "fixed", "mid", "long"])
def test_shared_rcs_parity(kind):
    s, uv, P = _case(kind)
    lam = 1e-3
    S, b, F_ref = P.rcs(s.ext_init, s.intr_init, s.pts_init, lam)
    rp_ref, ci_ref, blk_ref, rhs_ref = P.padded_blocks(S, b)
    ctx = _ctx(s, uv)
    try:
        F = ba.ba_linearize(ctx, _params(s.ext_init, s.intr_init), T(s.pts_init, torch.float64))
        ba.ba_form_rcs(ctx, lam)
        rp, ci = ba.ba_get_pattern(ctx)
        blk, rhs = ba.ba_get_rcs(ctx)
    finally:
        ba.ba_destroy(ctx)
    assert np.array_equal(rp, rp_ref) and np.array_equal(ci, ci_ref)
    assert abs(F - F_ref) <= 1e-11 * F_ref
    errs, raw = block_errors(blk, blk_ref, rp_ref, ci_ref)
    assert errs.max() <= 1e-10, (errs.max(), raw.max())
    rerr = np.linalg.norm(rhs - rhs_ref, axis=1) / np.maximum(np.linalg.norm(rhs_ref, axis=1), 1e-300)
    assert rerr.max() <= 1e-9
    for u in range(len(rp) - 1):
        nreal = 6 if u < P.n_free else 5
        d = blk[rp[u]]
        assert np.array_equal(d, d.T)
        assert np.array_equal(d[nreal:, nreal:], np.eye(9 - nreal)) and not d[nreal:, :nreal].any()
        assert not rhs[u, nreal:].any()


def test_shared_pcg_solution():
    s, uv, P = _case("mid")
    S, b, _ = P.rcs(s.ext_init, s.intr_init, s.pts_init, 1e-3)
    x_ref = np.linalg.solve(S, b)
    node, slot = P.nodes_of_unknowns()
    ctx = _ctx(s, uv)
    try:
        ba.ba_linearize(ctx, _params(s.ext_init, s.intr_init), T(s.pts_init, torch.float64))
        ba.ba_form_rcs(ctx, 1e-3)
        n_rows = ba.ba_get_sizes(ctx)["n_rows"]
        dx = torch.empty((n_rows, 9), dtype=torch.float64, device="cuda")
        for pre in (ba.BA_PRECOND_BLOCK_JACOBI, ba.BA_PRECOND_FSAI):
            info = ba.ba_pcg_solve(ctx, dx, tol=1e-12, max_iter=20000, precond=pre)
            assert info["status"] == 0
            x = dx.cpu().numpy()
            assert np.linalg.norm(x[node, slot] - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
            pad = np.ones_like(x, bool)
            pad[node, slot] = False
            assert not x[pad].any()
        with pytest.raises(ba.BAError):
            ba.ba_pcg_solve(ctx, dx, deflate=True)
    finally:
        ba.ba_destroy(ctx)


@pytest.mark.parametrize("kind", ["small", "long_small"])
def test_shared_lm_step_and_trajectory(kind):
    s, uv, P = _case(kind)
    ctx = _ctx(s, uv)
    try:
        # one step with the RCS solved tightly: the dense step of Eq. (1)
        params = _params(s.ext_init, s.intr_init)
        pts = T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        info = ba.ba_lm_step(ctx, params, pts, st, pcg_tol=1e-12, pcg_max_iter=20000)
        de, dq, dp, F, pred = P.dense_step(s.ext_init, s.intr_init, s.pts_init, 1e-4)
        Fn_ref = P.cost(s.ext_init + de, s.intr_init + dq, s.pts_init + dp)
        assert info["accepted"] == 1
        assert abs(info["cost"] - F) <= 1e-11 * F
        assert abs(info["model_decrease"] - pred) <= 1e-8 * abs(pred)
        assert abs(info["cost_new"] - Fn_ref) <= 1e-8 * Fn_ref
        pv = params.cpu().numpy()
        ext1 = pv[:6 * s.n_img].reshape(-1, 6)
        intr1 = pv[6 * s.n_img:].reshape(-1, 5)
        assert np.abs(ext1 - (s.ext_init + de)).max() <= 1e-8 * np.abs(de).max()
        assert np.abs(intr1 - (s.intr_init + dq)).max() <= 1e-8 * np.abs(dq).max()
        assert np.abs(pts.cpu().numpy() - (s.pts_init + dp)).max() <= 1e-8 * np.abs(dp).max()
    finally:
        ba.ba_destroy(ctx)
    # 8 iterations from the start against the reference's LM
    _, _, _, hist_ref = I.lm_run(P, s.ext_init, s.intr_init, s.pts_init, 8)
    ctx = _ctx(s, uv)
    try:
        params = _params(s.ext_init, s.intr_init)
        pts = T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        hist = [ba.ba_lm_step(ctx, params, pts, st, pcg_tol=1e-10, pcg_max_iter=20000) for _ in range(8)]
        pv = params.cpu().numpy()
        F_fin = P.cost(pv[:6 * s.n_img].reshape(-1, 6), pv[6 * s.n_img:].reshape(-1, 5), pts.cpu().numpy())
    finally:
        ba.ba_destroy(ctx)
    for h, r in zip(hist, hist_ref):
        if abs(r["cost"] - r["cost_new"]) > 1e-8 * r["cost"]:
            assert h["accepted"] == r["accepted"]
            assert abs(h["cost"] - r["cost"]) <= 1e-6 * r["cost"]
    F_ref_fin = min(r["cost_new"] if r["accepted"] else r["cost"] for r in hist_ref)
    assert abs(F_fin - F_ref_fin) <= 1e-6 * F_ref_fin


def test_shared_invalid_inputs():
    s, uv, P = _case("small")
    bad = s.img_cam.copy()
    bad[2] = s.n_phys
    with pytest.raises(ba.BAError) as ei:
        ba.ba_create_shared(s.n_img, s.n_phys, s.n_pts, T(s.obs_img, torch.int32), T(s.obs_pt, torch.int32),
                            T(uv, torch.float64), T(bad, torch.int32))
    assert ei.value.status == ba.BA_ERR_INVALID_ARG
    ctx = _ctx(s, uv)
    try:
        params = _params(s.ext_init, s.intr_init)
        pts = T(s.pts_init, torch.float64)
        with pytest.raises(ba.BAError):
            ba.ba_triangulate(ctx, params, pts)
        with pytest.raises(ba.BAError):
            ba.ba_lm_step(ctx, params, pts, ba.new_lm_state(1e-4), retriangulate=2)
        ba.ba_linearize(ctx, params, pts)
        with pytest.raises(ba.BAError):
            ba.ba_get_jacobians(ctx)
    finally:
        ba.ba_destroy(ctx)
