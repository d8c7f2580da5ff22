"""FSAI preconditioner on the GPU against the oracle (needs a GPU): the
factor G of the current RCS block by block, PCG solutions and iteration
counts, and LM runs with the FSAI preconditioner."""
import numpy as np
import pytest

from oracle import fsai
from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from gpu_util import T, create

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")

CAP = 27   # lower neighbours kept per row by the library


def _case(scene, lam=1e-3, precision=0):
    uv = orc.observations(scene)
    P = orc.Problem.from_scene(scene, uv)
    P.linearize(scene.cams_init, scene.pts_init)
    P.form_rcs(lam)
    ctx = create(scene, uv, precision)
    ba.ba_linearize(ctx, T(scene.cams_init, torch.float64), T(scene.pts_init, torch.float64))
    ba.ba_form_rcs(ctx, lam)
    return P, ctx


def _oracle_fsai(P, scene):
    blk, rhs = P.rcs()
    rp, ci = P.pattern()
    cnt = fsai.shared_points(P.n_rows, P.cam_row(), scene.obs_cam, scene.obs_pt)
    G, Gs, J = fsai.fsai(blk, rp, ci, cnt, cap=CAP)
    return blk, rhs, rp, ci, G, Gs, J


def _dense_scene():
    # 49 cameras, every point seen by up to 10 random cameras: rows have
    # more than CAP lower neighbours, so the common-point rule decides
    return scenegen.tiny_scene(seed=5, n_grid=7, n_pts=3000, t_hi=10, with_stats=False)


@pytest.mark.parametrize("kind", ["grid", "dense"])
def test_fsai_factor_parity(kind):
    s = (scenegen.aerial_grid_scene(seed=4, nx=10, ny=8, n_pts=12000, with_stats=False)
         if kind == "grid" else _dense_scene())
    P, ctx = _case(s)
    try:
        n_rows = P.n_rows
        dxc = torch.empty((n_rows, 9), dtype=torch.float64, device="cuda")
        info = ba.ba_pcg_solve(ctx, dxc, tol=1e-10, max_iter=3000, precond=ba.BA_PRECOND_FSAI)
        assert info["status"] == 0
        Gg = ba.ba_get_fsai(ctx).astype(np.float64)
    finally:
        ba.ba_destroy(ctx)
    blk, rhs, rp, ci, G, Gs, J = _oracle_fsai(P, s)
    if kind == "dense":
        assert max(len(j) for j in J) == CAP + 1
        assert sum(1 for r in range(n_rows) for k in range(rp[r] + 1, rp[r + 1])) > n_rows * CAP / 2
    nz = np.array([np.abs(g).max() > 0 for g in Gs])
    # slots of dropped neighbours are exactly zero on both sides
    assert np.array_equal(nz, np.array([np.abs(g).max() > 0 for g in Gg]))
    # FP32 local factorisation: relative block error (Frobenius) <= 1e-4
    err = np.array([np.linalg.norm(Gg[k] - Gs[k]) / np.linalg.norm(Gs[k]) for k in np.flatnonzero(nz)])
    assert err.max() <= 1e-4, err.max()


def test_fsai_pcg_parity():
    s = scenegen.aerial_grid_scene(seed=4, nx=10, ny=8, n_pts=12000, with_stats=False)
    P, ctx = _case(s)
    try:
        dxc = torch.empty((P.n_rows, 9), dtype=torch.float64, device="cuda")
        info = ba.ba_pcg_solve(ctx, dxc, tol=1e-12, max_iter=5000, precond=ba.BA_PRECOND_FSAI)
        x = dxc.cpu().numpy()
        info6 = ba.ba_pcg_solve(ctx, dxc, tol=1e-6, precond=ba.BA_PRECOND_FSAI)
        x6 = dxc.cpu().numpy()
        bj6 = ba.ba_pcg_solve(ctx, dxc, tol=1e-6)
    finally:
        ba.ba_destroy(ctx)
    blk, rhs, rp, ci, G, Gs, J = _oracle_fsai(P, s)
    S = fsai.dense_rcs(blk, rp, ci)
    b = rhs.ravel()
    x_ref = np.linalg.solve(S, b)
    assert info["status"] == 0 and info["relres"] <= 1e-12
    np.testing.assert_allclose(x.ravel(), x_ref, rtol=0, atol=1e-7 * np.abs(x_ref).max())
    # iteration counts against the oracle's FSAI PCG (FP64 factor)
    _, it_ref, _ = fsai.pcg(lambda v: S @ v, b, lambda v: G.T @ (G @ v), tol=1e-12, max_iter=5000)
    assert abs(info["iters"] - it_ref) <= max(3, 0.1 * it_ref)
    _, it6_ref, _ = fsai.pcg(lambda v: S @ v, b, lambda v: G.T @ (G @ v), tol=1e-6, max_iter=1000)
    assert info6["status"] == 0 and abs(info6["iters"] - it6_ref) <= max(3, 0.1 * it6_ref)
    assert np.linalg.norm(b - S @ x6.ravel()) <= 1.5e-6 * np.linalg.norm(b)
    # the factorised preconditioner needs fewer iterations than block-Jacobi
    assert info6["iters"] < bj6["iters"]


@pytest.mark.parametrize("kind", ["grid", "dense"])
def test_fsai_in_both_product_layouts(kind):
    """Exact FSAI applied with the FULL layout (FP32 blocks of G and G^T by
    rows) and with the UPPER layout (the FP16 copy of the Jacobi-scaled
    factor, one 16-byte group plus one half per column): iteration counts
    equal up to the FP16 rounding of the factor, and both solutions within
    1e-7 of the oracle's solve."""
    s = (scenegen.aerial_grid_scene(seed=7, nx=10, ny=8, n_pts=12000, with_stats=False)
         if kind == "grid" else _dense_scene())
    P, ctx = _case(s)
    try:
        dxc = torch.empty((P.n_rows, 9), dtype=torch.float64, device="cuda")
        out = {}
        for prod in (ba.BA_PRODUCT_FULL, ba.BA_PRODUCT_UPPER, ba.BA_PRODUCT_UPPER):
            info = ba.ba_pcg_solve(ctx, dxc, tol=1e-10, max_iter=5000, precond=ba.BA_PRECOND_FSAI, product=prod)
            assert info["status"] == 0
            out.setdefault(prod, []).append((info["iters"], dxc.cpu().numpy().copy()))
    finally:
        ba.ba_destroy(ctx)
    (i_f, x_f), = out[ba.BA_PRODUCT_FULL]
    (i_u, x_u), (i_u2, x_u2) = out[ba.BA_PRODUCT_UPPER]
    # the FP16 copy is made once per RCS: a second solve repeats the first
    assert i_u2 == i_u and np.array_equal(x_u2, x_u)
    assert abs(i_u - i_f) <= max(2, 0.05 * i_f)
    x_ref, _ = P.pcg(tol=1e-12, max_iter=5000)
    for xv in (x_f, x_u):
        assert np.linalg.norm(xv - x_ref) <= 1e-7 * np.linalg.norm(x_ref)


def test_fsai_initial_guess_and_reuse():
    s = scenegen.aerial_grid_scene(seed=6, nx=8, ny=6, n_pts=6000, with_stats=False)
    P, ctx = _case(s)
    try:
        x_ref, _ = P.pcg(tol=1e-12, max_iter=5000)
        dxc = torch.empty((P.n_rows, 9), dtype=torch.float64, device="cuda")
        a = ba.ba_pcg_solve(ctx, dxc, tol=1e-8, precond=ba.BA_PRECOND_FSAI)
        xa = dxc.cpu().numpy().copy()
        b = ba.ba_pcg_solve(ctx, dxc, tol=1e-8, precond=ba.BA_PRECOND_FSAI, x0=torch.zeros_like(dxc))
        assert a["iters"] == b["iters"] and np.array_equal(xa, dxc.cpu().numpy())
        ba.ba_pcg_solve(ctx, dxc, tol=1e-3, precond=ba.BA_PRECOND_FSAI)
        warm = dxc.clone()
        c = ba.ba_pcg_solve(ctx, dxc, tol=1e-9, precond=ba.BA_PRECOND_FSAI, x0=warm)
        assert c["status"] == 0
        assert np.linalg.norm(dxc.cpu().numpy() - x_ref) <= 1e-6 * np.linalg.norm(x_ref)
        # block-Jacobi after FSAI on the same context is unchanged
        d = ba.ba_pcg_solve(ctx, dxc, tol=1e-8)
        _, oinfo = P.pcg(tol=1e-8)
        assert abs(d["iters"] - oinfo["iters"]) <= max(3, 0.1 * oinfo["iters"])
        info = ba.ba_pcg_solve(ctx, dxc, tol=1e-12, max_iter=3, precond=ba.BA_PRECOND_FSAI)
        assert info["status"] == ba.BA_ERR_NOT_CONVERGED and info["iters"] == 3
    finally:
        ba.ba_destroy(ctx)


@pytest.mark.parametrize("precision", [0, 1])
def test_lm_with_fsai_final_cost(precision):
    s = scenegen.aerial_grid_scene(seed=7, nx=8, ny=6, n_pts=6000, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    c_ref, p_ref, _ = orc.lm_run(P, s.cams_init, s.pts_init, 10)
    F_ref = P.cost(c_ref, p_ref)
    ctx = create(s, uv, precision)
    try:
        cams = T(s.cams_init, torch.float64)
        pts = T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        for _ in range(10):
            info = ba.ba_lm_step(ctx, cams, pts, st, precond=ba.BA_PRECOND_FSAI)
            assert info["pcg_status"] in (0, ba.BA_ERR_NOT_CONVERGED)
        F = P.cost(cams.cpu().numpy(), pts.cpu().numpy())
    finally:
        ba.ba_destroy(ctx)
    assert abs(F - F_ref) <= 1e-6 * F_ref
