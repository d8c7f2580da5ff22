"""HIP path against the oracle on identical seeded inputs (needs a GPU).

Bars: pattern bit-exact; Jacobians / residuals to ~1e-12; RCS blocks to
1e-10 (FP64) and 1e-4 (mixed) in the floored per-block metric; PCG
solution, back-substitution and LM trajectory; final cost to rel 1e-6."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from conftest import small_scene
from gpu_util import T, block_errors, create

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")


def _mid_scene(seed=4, n_pts=20000):
    # 10 x 8 grid: several tiles of every kernel plus ragged tails
    return scenegen.aerial_grid_scene(seed=seed, nx=10, ny=8, n_pts=n_pts, with_stats=False)


def _both(scene, uv=None, precision=0, lam=1e-4, params="init"):
    uv = orc.observations(scene) if uv is None else uv
    cams = scene.cams_init if params == "init" else scene.cams_true
    pts = scene.pts_init if params == "init" else scene.pts_true
    P = orc.Problem.from_scene(scene, uv)
    F_ref = P.linearize(cams, pts)
    P.form_rcs(lam)
    ctx = create(scene, uv, precision)
    F = ba.ba_linearize(ctx, T(cams, torch.float64), T(pts, torch.float64))
    ba.ba_form_rcs(ctx, lam)
    return P, F_ref, ctx, F


@pytest.mark.parametrize("variant", ["plain", "fixed", "shuffled"])
def test_pattern_bit_exact(variant):
    s = scenegen.tiny_scene(seed=7, n_pts=300, with_stats=False)
    uv = orc.observations(s)
    if variant == "fixed":
        s.cam_fixed[[2, 5, 11]] = 1
    if variant == "shuffled":
        s, perm = scenegen.shuffled(s)
        uv = uv[:, perm]
    P = orc.Problem.from_scene(s, uv)
    ctx = create(s, uv)
    try:
        rp, ci = ba.ba_get_pattern(ctx)
        rp_ref, ci_ref = P.pattern()
        assert np.array_equal(rp, rp_ref) and np.array_equal(ci, ci_ref)
    finally:
        ba.ba_destroy(ctx)


def test_project_matches_oracle():
    s = _mid_scene(n_pts=5000)
    uv_ref = orc.observations(s)
    uv = ba.ba_project(T(s.cams_true, torch.float64), T(s.pts_true, torch.float64),
                       T(s.obs_cam, torch.int32), T(s.obs_pt, torch.int32), T(s.noise, torch.float64))
    np.testing.assert_allclose(uv.cpu().numpy(), uv_ref, rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("theta_mode", ["nadir", "small"])
def test_linearize_parity(theta_mode):
    s = small_scene(seed=11, n_pts=200)
    if theta_mode == "small":
        # rotations near zero (series branch of the closed-form Jacobian)
        # (t keeps P_z = X_z + 10 > 0 once R is close to the identity)
        s.cams_init[:, :3] *= 1e-3 / np.linalg.norm(s.cams_init[:, :3], axis=1, keepdims=True)
    uv = orc.observations(s)
    F_ref, e_ref, Jc, Jp = orc.linearize(s.cams_init, s.pts_init, s.obs_cam, s.obs_pt, uv)
    ctx = create(s, uv)
    try:
        F = ba.ba_linearize(ctx, T(s.cams_init, torch.float64), T(s.pts_init, torch.float64))
        J, e = ba.ba_get_jacobians(ctx)
        J_ref = np.concatenate([Jc.reshape(-1, 18), Jp.reshape(-1, 6)], axis=1)
        scale = np.abs(J_ref).max(axis=1, keepdims=True)
        assert (np.abs(J - J_ref) / scale).max() <= 1e-11
        np.testing.assert_allclose(e, e_ref, rtol=0, atol=1e-9)
        assert abs(F - F_ref) <= 1e-11 * F_ref
    finally:
        ba.ba_destroy(ctx)


def test_zero_residual_noise_free():
    s = _mid_scene(n_pts=4000)
    uv = orc.project(s.cams_true, s.pts_true, s.obs_cam, s.obs_pt)
    ctx = create(s, uv)
    try:
        F = ba.ba_linearize(ctx, T(s.cams_true, torch.float64), T(s.pts_true, torch.float64))
        _, e = ba.ba_get_jacobians(ctx)
        assert np.abs(e).max() < 1e-9 and F < 1e-18 * s.n_obs
    finally:
        ba.ba_destroy(ctx)


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-4)])
@pytest.mark.parametrize("scene_kind", ["tiny", "mid", "fixed"])
def test_rcs_parity(precision, tol, scene_kind):
    if scene_kind == "tiny":
        s = scenegen.tiny_scene(seed=0, with_stats=False)
    else:
        s = _mid_scene()
        if scene_kind == "fixed":
            s.cam_fixed[[0, 9, 40, 79]] = 1
    for lam in (1e-4, 0.5):
        P, F_ref, ctx, F = _both(s, precision=precision, lam=lam)
        try:
            blk, rhs = ba.ba_get_rcs(ctx)
            blk_ref, rhs_ref = P.rcs()
            rp, ci = P.pattern()
            errs, raw = block_errors(blk, blk_ref, rp, ci)
            assert errs.max() <= tol, (errs.max(), np.quantile(errs, 0.999), raw.max())
            rerr = np.linalg.norm(rhs - rhs_ref, axis=1) / np.maximum(np.linalg.norm(rhs_ref, axis=1), 1e-300)
            assert rerr.max() <= (1e-9 if precision == 0 else 1e-4), rerr.max()
            # diagonal blocks are exactly symmetric
            for r in range(len(rp) - 1):
                assert np.array_equal(blk[rp[r]], blk[rp[r]].T)
            assert abs(F - F_ref) <= 1e-11 * F_ref
        finally:
            ba.ba_destroy(ctx)


def test_rcs_deterministic():
    s = _mid_scene(n_pts=8000)
    P, _, ctx, _ = _both(s)
    try:
        a = ba.ba_get_rcs(ctx)
        ba.ba_form_rcs(ctx, 1e-4)
        b = ba.ba_get_rcs(ctx)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    finally:
        ba.ba_destroy(ctx)


def test_pcg_and_back_substitution_parity():
    s = _mid_scene(n_pts=10000)
    P, _, ctx, _ = _both(s, lam=1e-3)
    try:
        n_rows = P.n_rows
        dxc = torch.empty((n_rows, 9), dtype=torch.float64, device="cuda")
        info = ba.ba_pcg_solve(ctx, dxc, tol=1e-12, max_iter=5000)
        x_ref, oinfo = P.pcg(tol=1e-12, max_iter=5000)
        x = dxc.cpu().numpy()
        assert info["status"] == 0 and info["relres"] <= 1e-12
        assert np.linalg.norm(x - x_ref) <= 1e-7 * np.linalg.norm(x_ref)
        assert abs(info["iters"] - oinfo["iters"]) <= max(3, 0.05 * oinfo["iters"])
        # same tolerance as the LM path: near the stop threshold the residual
        # plateaus, so rounding may move the stopping step by a few; the GPU
        # solution must meet the tolerance in the oracle's own product
        info6 = ba.ba_pcg_solve(ctx, dxc, tol=1e-6)
        _, oinfo6 = P.pcg(tol=1e-6)
        assert info6["status"] == 0 and info6["relres"] <= 1e-6
        assert abs(info6["iters"] - oinfo6["iters"]) <= max(3, 0.1 * oinfo6["iters"])
        _, rhs_ref = P.rcs()
        true_res = np.linalg.norm(rhs_ref - P.spmv(dxc.cpu().numpy())) / np.linalg.norm(rhs_ref)
        assert true_res <= 1.5e-6, true_res
        # back-substitution from the same dxc
        dxc_t = T(x_ref, torch.float64)
        dxp = torch.empty((s.n_pts, 3), dtype=torch.float64, device="cuda")
        ba.ba_back_substitute(ctx, dxc_t, dxp)
        dxp_ref = P.back_substitute(x_ref)
        np.testing.assert_allclose(dxp.cpu().numpy(), dxp_ref, rtol=0, atol=1e-10 * np.abs(dxp_ref).max())
    finally:
        ba.ba_destroy(ctx)


def test_pcg_initial_guess_and_limits():
    s = _mid_scene(n_pts=6000)
    P, _, ctx, _ = _both(s, lam=1e-3)
    try:
        x_ref, _ = P.pcg(tol=1e-12, max_iter=5000)
        dxc = torch.empty((P.n_rows, 9), dtype=torch.float64, device="cuda")
        a = ba.ba_pcg_solve(ctx, dxc, tol=1e-8)
        xa = dxc.cpu().numpy().copy()
        # an explicit zero initial guess is the default start, bit for bit
        b = ba.ba_pcg_solve(ctx, dxc, tol=1e-8, x0=torch.zeros_like(dxc))
        assert a["iters"] == b["iters"] and np.array_equal(xa, dxc.cpu().numpy())
        # warm start from a loose solution still reaches the solution
        ba.ba_pcg_solve(ctx, dxc, tol=1e-3)
        warm = dxc.clone()
        c = ba.ba_pcg_solve(ctx, dxc, tol=1e-9, x0=warm)
        assert c["status"] == 0
        assert np.linalg.norm(dxc.cpu().numpy() - x_ref) <= 1e-6 * np.linalg.norm(x_ref)
        info = ba.ba_pcg_solve(ctx, dxc, tol=1e-12, max_iter=3)
        assert info["status"] == ba.BA_ERR_NOT_CONVERGED and info["iters"] == 3
        info = ba.ba_pcg_solve(ctx, dxc, tol=1e-12, max_iter=0)
        assert info["iters"] == 0
    finally:
        ba.ba_destroy(ctx)


@pytest.mark.parametrize("precision", [0, 1])
def test_lm_trajectory(precision):
    s = scenegen.tiny_scene(seed=0, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    _, _, hist_ref = orc.lm_run(P, s.cams_init, s.pts_init, 10)
    ctx = create(s, uv, precision)
    try:
        cams = T(s.cams_init, torch.float64)
        pts = T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        hist = []
        for _ in range(10):
            lam0, nu0 = st.lam, st.nu
            h = ba.ba_lm_step(ctx, cams, pts, st)
            h.update(lam_factor=st.lam / lam0, nu_after=st.nu, nu_before=nu0)
            hist.append(h)
        # each step solves the RCS only to PCG rel 1e-6, so iterates agree to
        # about that level; the cost of each iterate is compared at 1e-6
        tol = 1e-6 if precision == 0 else 1e-5
        lam_prev, nu_ref = 1e-4, 2.0
        n_acc = n_rej = 0
        in_sync = True   # every earlier decision agreed (a tie may go either way)
        for h, r in zip(hist, hist_ref):
            # oracle's damping factor of this step and its nu afterwards
            r_factor = r["lambda_after"] / lam_prev
            lam_prev = r["lambda_after"]
            nu_ref_before = nu_ref
            nu_ref = 2.0 if r["accepted"] else 2.0 * nu_ref
            # decisions (accept and reject) are compared while the step is far
            # from a tie
            if abs(r["cost"] - r["cost_new"]) > 1e-8 * r["cost"]:
                assert h["accepted"] == r["accepted"]
                assert abs(h["cost"] - r["cost"]) <= tol * r["cost"]
            if h["accepted"] != r["accepted"]:
                in_sync = False
            if in_sync and abs(r["cost"] - r["cost_new"]) > 1e-8 * r["cost"]:
                assert h["nu_before"] == nu_ref_before and h["nu_after"] == nu_ref
                if r["accepted"]:
                    n_acc += 1
                    # lambda *= max(1/3, 1 - (2 rho - 1)^3): compared where the
                    # gain ratio is well resolved by both sides' costs
                    if r["cost"] - r["cost_new"] > 1e-4 * r["cost"]:
                        assert h["lam_factor"] == pytest.approx(r_factor, rel=1e-3 if precision == 0 else 1e-2)
                else:
                    n_rej += 1
                    assert h["lam_factor"] == r_factor == nu_ref_before
        assert n_acc >= 3
        F_fin = min(h["cost_new"] if h["accepted"] else h["cost"] for h in hist)
        F_ref_fin = min(h["cost_new"] if h["accepted"] else h["cost"] for h in hist_ref)
        assert abs(F_fin - F_ref_fin) <= 1e-6 * F_ref_fin
    finally:
        ba.ba_destroy(ctx)


def test_lm_mid_scene_final_cost():
    s = _mid_scene(n_pts=20000)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    c_ref, p_ref, hist_ref = orc.lm_run(P, s.cams_init, s.pts_init, 8)
    ctx = create(s, uv)
    try:
        cams = T(s.cams_init, torch.float64)
        pts = T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        for _ in range(8):
            ba.ba_lm_step(ctx, cams, pts, st)
        F = P.cost(cams.cpu().numpy(), pts.cpu().numpy())
        F_ref = P.cost(c_ref, p_ref)
        assert abs(F - F_ref) <= 1e-6 * F_ref
    finally:
        ba.ba_destroy(ctx)


def test_reject_keeps_parameters():
    """A start far outside the region where the quadratic model holds (points
    pulled 3.5 units towards the cameras and scattered, lambda ~ 0): the oracle
    rejects with F' well above F, so must the library; parameters then stay
    bitwise unchanged and lambda *= nu, nu *= 2."""
    s = scenegen.tiny_scene(seed=2, with_stats=False)
    uv = orc.observations(s)
    rng = np.random.default_rng(0)
    pts0 = s.pts_true.copy()
    pts0[:, 2] = 6.0
    pts0[:, :2] += rng.normal(0, 2.0, (s.n_pts, 2))
    P = orc.Problem.from_scene(s, uv)
    ost = orc.LMState(lam=1e-12, nu=2.0, iter=0, pad=0)
    oinfo = P.lm_step(s.cams_true.copy(), pts0.copy(), ost)
    assert oinfo["accepted"] == 0 and oinfo["cost_new"] > 1.2 * oinfo["cost"]
    ctx = create(s, uv)
    try:
        cams = T(s.cams_true, torch.float64)
        pts = T(pts0, torch.float64)
        st = ba.new_lm_state(1e-12)
        info = ba.ba_lm_step(ctx, cams, pts, st)
        assert info["accepted"] == 0 and st.flags & 1
        assert abs(info["cost"] - oinfo["cost"]) <= 1e-10 * oinfo["cost"]
        assert np.array_equal(cams.cpu().numpy(), s.cams_true) and np.array_equal(pts.cpu().numpy(), pts0)
        assert st.lam == pytest.approx(2e-12) and st.nu == 4.0 and st.iter == 1
        # the second attempt reuses the linearization (flag bit 0 set)
        info2 = ba.ba_lm_step(ctx, cams, pts, st)
        assert info2["cost"] == info["cost"] and st.iter == 2
    finally:
        ba.ba_destroy(ctx)


def test_invalid_inputs():
    s = small_scene(seed=1)
    uv = orc.observations(s)
    bad = s.obs_cam.copy(); bad[0] = s.n_cams
    import dataclasses
    with pytest.raises(ba.BAError) as ei:
        create(dataclasses.replace(s, obs_cam=bad), uv)
    assert ei.value.status == ba.BA_ERR_INVALID_ARG
    uvn = uv.copy(); uvn[1, 3] = np.nan
    with pytest.raises(ba.BAError):
        create(s, uvn)
    oc = np.concatenate([s.obs_cam, s.obs_cam[:1]]); op = np.concatenate([s.obs_pt, s.obs_pt[:1]])
    with pytest.raises(ba.BAError):
        create(dataclasses.replace(s, obs_cam=oc, obs_pt=op), np.concatenate([uv, uv[:, :1]], axis=1))
    ctx = create(s, uv)
    try:
        with pytest.raises(ba.BAError) as ei:
            ba.ba_form_rcs(ctx, 1e-3)
        assert ei.value.status == ba.BA_ERR_STATE
        ba.ba_linearize(ctx, T(s.cams_init, torch.float64), T(s.pts_init, torch.float64))
        with pytest.raises(ba.BAError):
            ba.ba_form_rcs(ctx, -1.0)
    finally:
        ba.ba_destroy(ctx)


@pytest.mark.parametrize("scene_kind", ["tiny", "fixed"])
def test_rcs_parity_undamped(scene_kind):
    """lambda = 0: the RCS is the Schur complement of J^T J itself (Eq. (4)
    without damping), positive semidefinite with the similarity gauge in its
    near-null space, so off-diagonal blocks cancel more than with damping;
    blocks and rhs against the oracle in the floored metric (the floor is
    what guards that cancellation)."""
    if scene_kind == "tiny":
        s = scenegen.tiny_scene(seed=0, with_stats=False)
    else:
        s = _mid_scene()
        s.cam_fixed[[0, 9, 40, 79]] = 1
    P, F_ref, ctx, F = _both(s, lam=0.0)
    try:
        blk, rhs = ba.ba_get_rcs(ctx)
        blk_ref, rhs_ref = P.rcs()
        rp, ci = P.pattern()
        errs, raw = block_errors(blk, blk_ref, rp, ci)
        assert errs.max() <= 1e-10, (errs.max(), raw.max())
        rerr = np.linalg.norm(rhs - rhs_ref, axis=1) / np.maximum(np.linalg.norm(rhs_ref, axis=1), 1e-300)
        assert rerr.max() <= 1e-9, rerr.max()
    finally:
        ba.ba_destroy(ctx)


def test_camera_without_observations():
    """A free camera that sees no point has a zero row in J: its diagonal
    RCS block is U* = (1 + lambda) 0 = 0, so formation reports
    BA_ERR_NOT_SPD (the oracle's block is zero too).  Fixed, the camera has
    no row, and the RCS equals the oracle's for the same observations."""
    import dataclasses
    s = scenegen.tiny_scene(seed=0, with_stats=False)
    uv = orc.observations(s)
    extra = s.cams_init[:1].copy()
    s2 = dataclasses.replace(s, n_cams=s.n_cams + 1, cams_true=np.concatenate([s.cams_true, extra]),
                             cams_init=np.concatenate([s.cams_init, extra]),
                             cam_fixed=np.concatenate([s.cam_fixed, np.zeros(1, np.uint8)]))
    P = orc.Problem.from_scene(s2, uv)
    P.linearize(s2.cams_init, s2.pts_init)
    P.form_rcs(1e-3)
    blk_ref, _ = P.rcs()
    rp, _ = P.pattern()
    assert not blk_ref[rp[s.n_cams]].any()
    ctx = create(s2, uv)
    try:
        ba.ba_linearize(ctx, T(s2.cams_init, torch.float64), T(s2.pts_init, torch.float64))
        with pytest.raises(ba.BAError) as ei:
            ba.ba_form_rcs(ctx, 1e-3)
        assert ei.value.status == ba.BA_ERR_NOT_SPD
    finally:
        ba.ba_destroy(ctx)
    s2.cam_fixed[s.n_cams] = 1
    P2, F_ref, ctx, F = _both(s2, uv=uv, lam=1e-3)
    try:
        blk, rhs = ba.ba_get_rcs(ctx)
        blk_ref, rhs_ref = P2.rcs()
        rp, ci = P2.pattern()
        errs, _ = block_errors(blk, blk_ref, rp, ci)
        assert len(rp) - 1 == s.n_cams and errs.max() <= 1e-10
        assert abs(F - F_ref) <= 1e-11 * F_ref
    finally:
        ba.ba_destroy(ctx)


def test_degenerate_observation_sets_rejected():
    """No observations, and a point seen once (its V_p has rank 2: Eq. (3)
    needs at least two views), are rejected at creation."""
    import dataclasses
    s = scenegen.tiny_scene(seed=0, with_stats=False)
    uv = orc.observations(s)
    with pytest.raises(ba.BAError) as ei:
        ba.ba_create(s.n_cams, s.n_pts, T(np.zeros(0, np.int32), torch.int32), T(np.zeros(0, np.int32), torch.int32),
                     T(np.zeros((2, 0)), torch.float64))
    assert ei.value.status == ba.BA_ERR_INVALID_ARG
    # point 0 keeps one observation
    first = np.flatnonzero(s.obs_pt == 0)
    keep = np.ones(s.n_obs, bool)
    keep[first[1:]] = False
    s1 = dataclasses.replace(s, obs_cam=s.obs_cam[keep], obs_pt=s.obs_pt[keep], n_obs=int(keep.sum()))
    with pytest.raises(ba.BAError) as ei:
        create(s1, uv[:, keep])
    assert ei.value.status == ba.BA_ERR_INVALID_ARG


def test_track_length_limits():
    """Contexts take tracks of any length: a point seen by more than 64
    cameras (one wave) goes to the workgroup-per-point kernels, with 9
    parameters per camera and with shared intrinsics."""
    import dataclasses
    s = scenegen.aerial_grid_scene(seed=3, nx=10, ny=8, n_pts=500, with_stats=False)
    uv = orc.observations(s)
    seen = set(s.obs_cam[s.obs_pt == 0].tolist())
    extra = [c for c in range(s.n_cams) if c not in seen][:65 - len(seen)]
    oc = np.concatenate([s.obs_cam, np.array(extra, np.int32)])
    op = np.concatenate([s.obs_pt, np.zeros(len(extra), np.int32)])
    uv2 = np.concatenate([uv, np.zeros((2, len(extra)))], axis=1)
    ba.ba_destroy(create(dataclasses.replace(s, obs_cam=oc, obs_pt=op, n_obs=len(oc)), uv2))
    sh = scenegen.shared_intrinsics_scene(seed=8, nx=10, ny=8, n_pts=500, n_phys=4)
    seen = set(sh.obs_img[sh.obs_pt == 0].tolist())
    extra = [c for c in range(sh.n_img) if c not in seen][:65 - len(seen)]
    oi = np.concatenate([sh.obs_img, np.array(extra, np.int32)])
    op = np.concatenate([sh.obs_pt, np.zeros(len(extra), np.int32)])
    ba.ba_destroy(ba.ba_create_shared(sh.n_img, sh.n_phys, sh.n_pts, T(oi, torch.int32), T(op, torch.int32),
                                      T(np.zeros((2, len(oi))), torch.float64), T(sh.img_cam, torch.int32), None))


def test_workspace_cap_out_of_memory():
    s = small_scene(seed=1)
    uv = orc.observations(s)
    from paper_2307_08383_amd import ba as b
    with pytest.raises(b.BAError) as ei:
        b.ba_create(s.n_cams, s.n_pts, T(s.obs_cam, torch.int32), T(s.obs_pt, torch.int32),
                    T(uv, torch.float64), workspace_cap=4096)
    assert ei.value.status == b.BA_ERR_OUT_OF_MEMORY


@pytest.mark.parametrize("precision", [0, 1])
def test_formation_not_spd(precision):
    """BA_ERR_NOT_SPD from formation.  A camera with focal length 0 has
    J_c = 0 in its rotation, translation and distortion columns (each carries
    the factor f), so its diagonal RCS block has zero rows; with every focal
    length 0 also J_p = 0, so every V_p is 0.  The oracle's U_ii, V_p agree
    (its formation fails on V_p, its diagonal block has a zero row).  An LM
    step on such an RCS is rejected and leaves the parameters unchanged."""
    s = scenegen.tiny_scene(seed=0, with_stats=False)
    uv = orc.observations(s)
    bad_cam = s.cams_init.copy()
    bad_cam[3, 6] = 0.0
    P = orc.Problem.from_scene(s, uv)
    P.linearize(bad_cam, s.pts_init)
    P.form_rcs(1e-4)
    blk_ref, _ = P.rcs()
    rp, _ = P.pattern()
    assert not np.any(blk_ref[rp[3]][0])   # zero row: not positive definite
    all_bad = s.cams_init.copy()
    all_bad[:, 6] = 0.0
    P.linearize(all_bad, s.pts_init)
    with pytest.raises(RuntimeError):
        P.form_rcs(1e-4)
    ctx = create(s, uv, precision)
    try:
        ba.ba_linearize(ctx, T(bad_cam, torch.float64), T(s.pts_init, torch.float64))
        with pytest.raises(ba.BAError) as ei:
            ba.ba_form_rcs(ctx, 1e-4)
        assert ei.value.status == ba.BA_ERR_NOT_SPD and "diagonal" in str(ei.value)
        ba.ba_linearize(ctx, T(all_bad, torch.float64), T(s.pts_init, torch.float64))
        with pytest.raises(ba.BAError) as ei:
            ba.ba_form_rcs(ctx, 1e-4)
        assert ei.value.status == ba.BA_ERR_NOT_SPD and "point" in str(ei.value)
        cams = T(bad_cam, torch.float64)
        pts = T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        info = ba.ba_lm_step(ctx, cams, pts, st, pcg_max_iter=50)
        assert info["accepted"] == 0 and info["pcg_status"] == ba.BA_ERR_NOT_SPD
        assert np.array_equal(cams.cpu().numpy(), bad_cam) and np.array_equal(pts.cpu().numpy(), s.pts_init)
    finally:
        ba.ba_destroy(ctx)


def test_mixed_records_out_of_range():
    """BA_ERR_RANGE: a point 1e-9 in front of a camera's image plane gives
    image coordinates near 1e9 and distortion derivatives near 1e48, beyond
    FP32 (3.4e38) but within FP64.  The FP64 path linearizes; the mixed path
    reports the overflow from ba_linearize, ba_form_rcs and ba_lm_step (no
    step, state unchanged)."""
    from scipy.spatial.transform import Rotation
    s = scenegen.tiny_scene(seed=0, with_stats=False)
    uv = orc.observations(s)
    c0, p0 = int(s.obs_cam[0]), int(s.obs_pt[0])
    R = Rotation.from_rotvec(s.cams_init[c0, :3]).as_matrix()
    pts0 = s.pts_init.copy()
    pts0[p0] = R.T @ (np.array([1.0, 0.5, 1e-9]) - s.cams_init[c0, 3:6])
    F_ref, e_ref, Jc, Jp = orc.linearize(s.cams_init, pts0, s.obs_cam, s.obs_pt, uv)
    assert np.isfinite(F_ref) and np.abs(Jc).max() > 1e40 and np.abs(Jc).max() < 1e300
    ctx = create(s, uv, 0)
    try:
        F = ba.ba_linearize(ctx, T(s.cams_init, torch.float64), T(pts0, torch.float64))
        # the camera-frame depth 1e-9 carries an absolute rounding error near
        # 1e-15 on either side, and F grows like depth^-10 here
        assert np.isfinite(F) and F == pytest.approx(F_ref, rel=1e-2)
    finally:
        ba.ba_destroy(ctx)
    ctx = create(s, uv, 1)
    try:
        cams = T(s.cams_init, torch.float64)
        pts = T(pts0, torch.float64)
        with pytest.raises(ba.BAError) as ei:
            ba.ba_linearize(ctx, cams, pts)
        assert ei.value.status == ba.BA_ERR_RANGE
        with pytest.raises(ba.BAError) as ei:
            ba.ba_form_rcs(ctx, 1e-4)
        assert ei.value.status == ba.BA_ERR_RANGE
        st = ba.new_lm_state(1e-4)
        with pytest.raises(ba.BAError) as ei:
            ba.ba_lm_step(ctx, cams, pts, st)
        assert ei.value.status == ba.BA_ERR_RANGE
        assert st.lam == 1e-4 and st.nu == 2.0 and st.iter == 0
        assert np.array_equal(cams.cpu().numpy(), s.cams_init) and np.array_equal(pts.cpu().numpy(), pts0)
    finally:
        ba.ba_destroy(ctx)
