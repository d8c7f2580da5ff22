"""PCG with an FP32 copy of the RCS for its products (solver_fp32), against
the CPU oracle (needs a GPU).  The solver then solves the system of the
rounded matrix exactly (FP64 vectors and recurrences); the LM run with it
reaches the oracle's final cost."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from gpu_util import T, create

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")


def _dense(blk, rp, ci, dtype):
    n = len(rp) - 1
    S = np.zeros((9 * n, 9 * n))
    for r in range(n):
        for k in range(rp[r], rp[r + 1]):
            c = ci[k]
            B = blk[k].astype(dtype).astype(np.float64)
            S[9 * r:9 * r + 9, 9 * c:9 * c + 9] = B
            if c != r:
                S[9 * c:9 * c + 9, 9 * r:9 * r + 9] = B.T
    return S


@pytest.mark.parametrize("deflate,precond", [(False, 0), (True, 0), (True, 2)])
def test_fp32_solver_solves_the_rounded_system(deflate, precond):
    s = scenegen.aerial_grid_scene(seed=4, nx=10, ny=8, n_pts=10000, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    P.linearize(s.cams_init, s.pts_init)
    P.form_rcs(1e-3)
    blk, rhs = P.rcs()
    rp, ci = P.pattern()
    S64 = _dense(blk, rp, ci, np.float64)
    S32 = _dense(blk, rp, ci, np.float32)
    b = rhs.ravel()
    ctx = create(s, uv, 0)
    try:
        ba.ba_linearize(ctx, T(s.cams_init, torch.float64), T(s.pts_init, torch.float64))
        ba.ba_form_rcs(ctx, 1e-3)
        dx = torch.empty((P.n_rows, 9), dtype=torch.float64, device="cuda")
        i64 = ba.ba_pcg_solve(ctx, dx, tol=1e-10, max_iter=5000, precond=precond, deflate=deflate)
        x64 = dx.cpu().numpy().ravel().copy()
        i32 = ba.ba_pcg_solve(ctx, dx, tol=1e-10, max_iter=5000, precond=precond, deflate=deflate, solver_fp32=True)
        x32 = dx.cpu().numpy().ravel().copy()
        # the FP64 solve again: the FP32 copy must not leak into it
        i64b = ba.ba_pcg_solve(ctx, dx, tol=1e-10, max_iter=5000, precond=precond, deflate=deflate)
        assert np.array_equal(dx.cpu().numpy().ravel(), x64) and i64b["iters"] == i64["iters"]
    finally:
        ba.ba_destroy(ctx)
    assert i64["status"] == 0 and i32["status"] == 0
    nb = np.linalg.norm(b)
    # the rounded system is solved (rare last-bit differences in the rounding
    # of blocks that differ from the oracle's in their last FP64 bits aside)
    assert np.linalg.norm(b - S32 @ x32) <= 1e-7 * nb
    # and the FP64 solution solves the FP64 system
    assert np.linalg.norm(b - S64 @ x64) <= 1e-9 * nb
    # the two solutions differ by the rounding of S, |dx| <= |S^-1| |dS| |x|,
    # plus what the two stopping tolerances leave (kappa * tol each)
    dS = np.linalg.norm(S64 - S32, 2)
    ev = np.linalg.eigvalsh(S64)
    nx = np.linalg.norm(x64)
    bound = 1.1 * dS / ev[0] * nx + 3.0 * (ev[-1] / ev[0]) * 1e-10 * nx
    assert np.linalg.norm(x32 - x64) <= bound


@pytest.mark.parametrize("precision", [0, 1])
def test_lm_with_fp32_solver_final_cost(precision):
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
            info = ba.ba_lm_step(ctx, cams, pts, st, precond=ba.BA_PRECOND_FSAI, deflate=True, solver_fp32=True)
            assert info["pcg_status"] in (0, ba.BA_ERR_NOT_CONVERGED)
        F = P.cost(cams.cpu().numpy(), pts.cpu().numpy())
    finally:
        ba.ba_destroy(ctx)
    assert abs(F - F_ref) <= 1e-6 * F_ref
