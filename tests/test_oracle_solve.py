"""Pins of the oracle's PCG, back-substitution and LM step (CPU only)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from conftest import small_scene
from test_oracle_rcs import dense_schur, dense_system, expand


def _problem(seed=5, lam=1e-3, fixed=None, noise=0.5, n_pts=60):
    s = small_scene(seed=seed, noise=noise, n_pts=n_pts)
    if fixed is not None:
        s.cam_fixed[fixed] = 1
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    P.linearize(s.cams_init, s.pts_init)
    P.form_rcs(lam)
    return s, P


def test_pcg_tight_tolerance_equals_cholesky_solve():
    s, P = _problem()
    blk, rhs = P.rcs()
    S = expand(P, blk)
    x_ref = np.linalg.solve(S, rhs.reshape(-1))
    x, info = P.pcg(tol=1e-14, max_iter=5000)
    assert info["status"] == 0 and info["relres"] <= 1e-14
    np.testing.assert_allclose(x.reshape(-1), x_ref, rtol=0, atol=1e-8 * np.abs(x_ref).max())


def test_pcg_relative_residual_reported():
    s, P = _problem()
    blk, rhs = P.rcs()
    S = expand(P, blk)
    x, info = P.pcg(tol=1e-6)
    r = rhs.reshape(-1) - S @ x.reshape(-1)
    rel = np.linalg.norm(r) / np.linalg.norm(rhs)
    assert info["status"] == 0
    assert rel <= 1.0000001e-6 and abs(rel - info["relres"]) <= 1e-9


def test_pcg_full_matrix_preconditioner_one_iteration():
    """M = S: M^-1 r0 is the solution, so one iteration converges (any S whose
    blocks are all on the diagonal, here by zeroing the off-diagonal blocks)."""
    s, P = _problem()
    blk, rhs = P.rcs()
    rp, ci = P.pattern()
    diag_only = np.zeros_like(blk)
    for r in range(P.n_rows):
        diag_only[rp[r]] = blk[rp[r]]
    P.set_rcs(diag_only, rhs)
    x, info = P.pcg(tol=1e-12)
    assert info["iters"] == 1 and info["status"] == 0
    for r in range(P.n_rows):
        np.testing.assert_allclose(blk[rp[r]] @ x[r], rhs[r], rtol=1e-10, atol=1e-10 * np.abs(rhs).max())


def test_pcg_explicit_preconditioner_and_limits():
    s, P = _problem()
    blk, rhs = P.rcs()
    rp, _ = P.pattern()
    M = np.stack([blk[rp[r]] for r in range(P.n_rows)])
    x1, i1 = P.pcg(tol=1e-8)
    x2, i2 = P.pcg(tol=1e-8, M=M)
    assert i1["iters"] == i2["iters"]
    np.testing.assert_allclose(x1, x2, rtol=0, atol=1e-12 * np.abs(x1).max())
    _, i3 = P.pcg(tol=1e-12, max_iter=2)
    assert i3["status"] == 4 and i3["iters"] == 2
    # CG terminates within the dimension in exact arithmetic; with rounding a
    # few more steps at most on this tiny, well-scaled system
    _, i4 = P.pcg(tol=1e-10, max_iter=10000)
    assert i4["iters"] <= 9 * P.n_rows + 20


def test_back_substitution_equals_dense_full_solve():
    """Eq. (4) + Eq. (5) reproduce the solution of the full damped system Eq. (1)."""
    for fixed in (None, [1]):
        lam = 2e-3
        s, P = _problem(lam=lam, fixed=fixed)
        J, Hs, g = dense_system(P, lam)
        full = np.linalg.solve(Hs, g)
        dxc, info = P.pcg(tol=1e-14, max_iter=5000)
        dxp = P.back_substitute(dxc)
        nc = 9 * P.n_rows
        np.testing.assert_allclose(dxc.reshape(-1), full[:nc], atol=1e-9 * np.abs(full).max())
        np.testing.assert_allclose(dxp.reshape(-1), full[nc:], atol=1e-9 * np.abs(full).max())
        # model terms from the stored J
        jdx2, dxl = P.model_terms(dxc, dxp)
        Jd = J @ full
        assert abs(jdx2 - Jd @ Jd) <= 1e-9 * (Jd @ Jd)
        assert abs(dxl - full @ g) <= 1e-9 * abs(full @ g)


def test_large_damping_gives_scaled_gradient_step():
    """lambda -> infinity: (J^T J + lambda diag(J^T J)) dx = g tends to
    dx = diag(J^T J)^-1 g / lambda (steepest descent with Marquardt scaling)."""
    lam = 1e9
    s, P = _problem(lam=lam)
    J, Hs, g = dense_system(P, lam)
    d = np.diag(J.T @ J)
    expect = g / (lam * d)
    dxc, _ = P.pcg(tol=1e-14, max_iter=5000)
    dxp = P.back_substitute(dxc)
    got = np.concatenate([dxc.reshape(-1), dxp.reshape(-1)])
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-5 * np.abs(expect).max())


def test_lm_noise_free_converges_to_zero_cost():
    s = scenegen.tiny_scene(seed=2, noise_sigma=0.0, with_stats=False)
    P = orc.Problem.from_scene(s)
    cams, pts, hist = orc.lm_run(P, s.cams_init, s.pts_init, 30, tol=1e-10)
    F = P.cost(cams, pts)
    rms = np.sqrt(2 * F / (2 * s.n_obs))
    assert rms < 1e-6, (rms, [h["cost"] for h in hist])


def test_lm_reaches_noise_floor():
    """With Gaussian pixel noise the optimum cost is about sigma^2/2 times the
    residual degrees of freedom (2 n_obs - unknowns + gauge)."""
    s = scenegen.tiny_scene(seed=0, with_stats=False)
    P = orc.Problem.from_scene(s)
    cams, pts, hist = orc.lm_run(P, s.cams_init, s.pts_init, 10)
    F = P.cost(cams, pts)
    dof = 2 * s.n_obs - 9 * s.n_cams - 3 * s.n_pts + 7
    expect = 0.5 * 0.25 * dof
    assert abs(F - expect) < 4 * 0.5 * 0.25 * np.sqrt(2 * dof)
    costs = [h["cost"] for h in hist]
    assert all(b <= a for a, b in zip(costs, costs[1:]))


def test_rejected_step_keeps_parameters_and_raises_damping():
    """At the exact optimum of noise-free data no step lowers the cost: the
    attempt is rejected, parameters stay bitwise equal and lambda *= nu,
    nu *= 2 (every attempt counts as an iteration)."""
    s = scenegen.tiny_scene(seed=2, noise_sigma=0.0, with_stats=False)
    P = orc.Problem.from_scene(s)
    cams = s.cams_true.copy(); pts = s.pts_true.copy()
    st = orc.LMState(lam=1e-3, nu=2.0, iter=0, pad=0)
    info = P.lm_step(cams, pts, st)
    assert info["accepted"] == 0
    assert np.array_equal(cams, s.cams_true) and np.array_equal(pts, s.pts_true)
    assert st.lam == pytest.approx(2e-3) and st.nu == 4.0 and st.iter == 1
    info = P.lm_step(cams, pts, st)
    assert st.lam == pytest.approx(8e-3) and st.nu == 8.0 and st.iter == 2


def test_accepted_step_nielsen_update():
    s = scenegen.tiny_scene(seed=0, with_stats=False)
    P = orc.Problem.from_scene(s)
    cams = s.cams_init.copy(); pts = s.pts_init.copy()
    st = orc.LMState(lam=1e-4, nu=8.0, iter=0, pad=0)
    info = P.lm_step(cams, pts, st)
    assert info["accepted"] == 1
    rho = info["rho"]
    assert st.lam == pytest.approx(1e-4 * max(1 / 3, 1 - (2 * rho - 1) ** 3))
    assert st.nu == 2.0
    assert P.cost(cams, pts) == pytest.approx(info["cost_new"], rel=1e-12)
