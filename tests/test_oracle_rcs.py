"""Pins of the oracle's pattern and reduced camera system (CPU only).

The RCS of Eq. (4) is the Schur complement of the damped normal matrix of
Eq. (1)/(3); these tests build that matrix densely from the Jacobian and
eliminate the points with LAPACK, independently of the oracle's
point-by-point formation (Sec. 5)."""
import itertools

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from conftest import small_scene


def dense_system(P: orc.Problem, lam):
    """Dense J (columns: free cameras by RCS row, then points), H* and g."""
    e, Jc, Jp = P.linearization()
    cam_row = P.cam_row()
    obs_cam, obs_pt = P._keep[0], P._keep[1]
    nr, npt = P.n_rows, P.n_pts
    J = np.zeros((2 * P.n_obs, 9 * nr + 3 * npt))
    for k in range(P.n_obs):
        r = cam_row[obs_cam[k]]
        if r >= 0:
            J[2 * k:2 * k + 2, 9 * r:9 * r + 9] = Jc[k]
        p = obs_pt[k]
        J[2 * k:2 * k + 2, 9 * nr + 3 * p:9 * nr + 3 * p + 3] = Jp[k]
    H = J.T @ J
    Hs = H + lam * np.diag(np.diag(H))
    g = -J.T @ e.reshape(-1)
    return J, Hs, g


def dense_schur(Hs, g, nc):
    Hcc, Hcp, Hpp = Hs[:nc, :nc], Hs[:nc, nc:], Hs[nc:, nc:]
    X = np.linalg.solve(Hpp, np.concatenate([Hcp.T, g[nc:, None]], axis=1))
    S = Hcc - Hcp @ X[:, :-1]
    b = g[:nc] - Hcp @ X[:, -1]
    return S, b


def expand(P: orc.Problem, blk):
    rp, ci = P.pattern()
    n = P.n_rows
    S = np.zeros((9 * n, 9 * n))
    for r in range(n):
        for k in range(rp[r], rp[r + 1]):
            s = ci[k]
            S[9 * r:9 * r + 9, 9 * s:9 * s + 9] = blk[k]
            if s != r:
                S[9 * s:9 * s + 9, 9 * r:9 * r + 9] = blk[k].T
    return S


def brute_pattern(n_cams, obs_cam, obs_pt, cam_fixed=None):
    rows = {}
    nr = 0
    for c in range(n_cams):
        if cam_fixed is None or not cam_fixed[c]:
            rows[c] = nr
            nr += 1
    tracks = {}
    for c, p in zip(obs_cam, obs_pt):
        tracks.setdefault(int(p), []).append(int(c))
    pairs = {(r, r) for r in range(nr)}
    for cams in tracks.values():
        for a, b in itertools.combinations(cams, 2):
            if a in rows and b in rows:
                ra, rb = rows[a], rows[b]
                pairs.add((min(ra, rb), max(ra, rb)))
    return nr, sorted(pairs)


@pytest.mark.parametrize("lam", [1e-4, 0.3])
@pytest.mark.parametrize("fixed", [False, True])
def test_rcs_equals_dense_schur(lam, fixed):
    s = small_scene(seed=5)
    if fixed:
        s.cam_fixed[[0, 4]] = 1
    uv = orc.observations(s, cams=s.cams_true, pts=s.pts_true)
    P = orc.Problem(s.n_cams, s.n_pts, s.obs_cam, s.obs_pt, uv, s.cam_fixed if fixed else None)
    P.linearize(s.cams_init, s.pts_init)
    P.form_rcs(lam)
    blk, rhs = P.rcs()
    _, Hs, g = dense_system(P, lam)
    S_ref, b_ref = dense_schur(Hs, g, 9 * P.n_rows)
    S = expand(P, blk)
    # the Schur complement of a symmetric matrix is symmetric
    assert np.abs(S_ref - S_ref.T).max() <= 1e-12 * np.abs(S_ref).max()
    np.testing.assert_allclose(S, S_ref, rtol=0, atol=1e-12 * np.abs(S_ref).max())
    np.testing.assert_allclose(rhs.reshape(-1), b_ref, rtol=0, atol=1e-11 * np.abs(b_ref).max())
    # per-block relative agreement
    rp, ci = P.pattern()
    for r in range(P.n_rows):
        for k in range(rp[r], rp[r + 1]):
            c = ci[k]
            ref = S_ref[9 * r:9 * r + 9, 9 * c:9 * c + 9]
            assert np.linalg.norm(blk[k] - ref) <= 1e-10 * max(np.linalg.norm(ref), 1e-3 * np.linalg.norm(S_ref[9 * r:9 * r + 9, 9 * r:9 * r + 9]))
    # damped RCS is positive definite
    assert np.linalg.eigvalsh(S).min() > 0


def test_rcs_psd_without_damping():
    """lambda = 0: S is a Schur complement of the PSD matrix J^T J, hence PSD;
    at the noise-free optimum the gauge freedom leaves a near-null space."""
    s = small_scene(seed=6, noise=0.0)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    P.linearize(s.cams_true, s.pts_true)
    P.form_rcs(0.0)
    S = expand(P, P.rcs()[0])
    ev = np.linalg.eigvalsh(S)
    assert ev.min() >= -1e-10 * ev.max()
    assert (ev < 1e-9 * ev.max()).sum() >= 6  # similarity gauge (7 dof, minus what the points absorb)


def test_pattern_matches_brute_force():
    s = scenegen.tiny_scene(seed=9, n_pts=200, with_stats=False)
    fixed = np.zeros(s.n_cams, np.uint8); fixed[[3, 7, 8]] = 1
    uv = orc.observations(s)
    for cf in (None, fixed):
        P = orc.Problem(s.n_cams, s.n_pts, s.obs_cam, s.obs_pt, uv, cf)
        nr, pairs = brute_pattern(s.n_cams, s.obs_cam, s.obs_pt, cf)
        rp, ci = P.pattern()
        got = [(r, int(ci[k])) for r in range(nr) for k in range(rp[r], rp[r + 1])]
        assert P.n_rows == nr and got == pairs
        # the diagonal block is first in each row
        assert all(ci[rp[r]] == r for r in range(nr))


def test_fig16_micro_example():
    """Five cameras; one point seen by cameras 1 and 3, one by 2 and 3 (Sec. 5,
    Fig. 16): the RCS has the diagonal plus blocks (1,3) and (2,3) only, and the
    point seen by 1 and 3 contributes S_13 = -W_1 V*^-1 W_3^T."""
    rng = np.random.default_rng(0)
    s = scenegen.tiny_scene(seed=1, n_pts=2, with_stats=False)
    cams = s.cams_true[:5].copy()
    obs_cam = np.array([0, 2, 1, 2], np.int32)
    obs_pt = np.array([0, 0, 1, 1], np.int32)
    pts = np.array([[5.0, 5.0, 0.5], [4.0, 6.0, 0.2]])
    uv = orc.project(cams, pts, obs_cam, obs_pt) + rng.normal(0, 0.5, (2, 4))
    P = orc.Problem(5, 2, obs_cam, obs_pt, uv)
    rp, ci = P.pattern()
    got = [(r, int(ci[k])) for r in range(5) for k in range(rp[r], rp[r + 1])]
    assert got == [(0, 0), (0, 2), (1, 1), (1, 2), (2, 2), (3, 3), (4, 4)]
    lam = 0.01
    P.linearize(cams, pts)
    P.form_rcs(lam)
    blk, _ = P.rcs()
    _, Hs, g = dense_system(P, lam)
    S_ref, _ = dense_schur(Hs, g, 45)
    np.testing.assert_allclose(blk[1], S_ref[0:9, 18:27], atol=1e-12 * np.abs(S_ref).max())
    # cameras 3 and 4 see nothing: their blocks are zero
    assert np.all(blk[5] == 0) and np.all(blk[6] == 0)


def test_point_groups_sum_to_global_rcs():
    """Sec. 5 / 6.1: the RCS is the sum of the sub-RCSs of any split of the
    points into groups."""
    s = small_scene(seed=8, n_pts=80)
    P = orc.Problem.from_scene(s)
    P.linearize(s.cams_init, s.pts_init)
    ref = None
    for G in (1, 2, 5, 13):
        P.form_rcs(1e-3, n_groups=G)
        blk, rhs = P.rcs()
        if ref is None:
            ref = (blk.copy(), rhs.copy())
        else:
            np.testing.assert_allclose(blk, ref[0], rtol=0, atol=1e-13 * np.abs(ref[0]).max())
            np.testing.assert_allclose(rhs, ref[1], rtol=0, atol=1e-12 * np.abs(ref[1]).max())


def test_observation_order_invariance():
    s = small_scene(seed=2)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    P.linearize(s.cams_init, s.pts_init); P.form_rcs(1e-3)
    blk, rhs = P.rcs()
    s2, perm = scenegen.shuffled(s)
    P2 = orc.Problem(s.n_cams, s.n_pts, s2.obs_cam, s2.obs_pt, uv[:, perm])
    P2.linearize(s.cams_init, s.pts_init); P2.form_rcs(1e-3)
    blk2, rhs2 = P2.rcs()
    np.testing.assert_allclose(blk2, blk, atol=1e-12 * np.abs(blk).max())
    np.testing.assert_allclose(rhs2, rhs, atol=1e-11 * np.abs(rhs).max())


def _dense_rcs(s, uv, lam):
    """S = H_cc - H_cp H_pp^-1 H_pc of the damped dense normal matrix,
    assembled from the per-observation Jacobian blocks (dense LAPACK)."""
    F, e, Jc, Jp = orc.linearize(s.cams_init, s.pts_init, s.obs_cam, s.obs_pt, uv)
    nc, npt = s.n_cams, s.n_pts
    J = np.zeros((2 * s.n_obs, 9 * nc + 3 * npt))
    for k in range(s.n_obs):
        c, p = s.obs_cam[k], s.obs_pt[k]
        J[2 * k:2 * k + 2, 9 * c:9 * c + 9] = Jc[k]
        J[2 * k:2 * k + 2, 9 * nc + 3 * p:9 * nc + 3 * p + 3] = Jp[k]
    H = J.T @ J
    H[np.diag_indices_from(H)] *= 1.0 + lam
    m = 9 * nc
    return H[:m, :m] - H[:m, m:] @ np.linalg.solve(H[m:, m:], H[m:, :m])


def test_bsmc_bytes_eq9():
    """Eq. (9) against an independent count.  The sparsity alpha is the
    fraction of non-zero 9x9 blocks (both triangles, with the diagonal) of
    the dense RCS built by dense elimination on the full normal matrix,
    without the oracle's pattern; the oracle's BSMC byte count must equal
    Eq. (9) evaluated with that alpha, for c = 9 and c = 11 unknowns per
    camera.  Eq. (10) is then checked against Y_C / Y_B of Eq. (8)-(9)
    (with its denominator term 3 alpha read as 3 alpha n)."""
    s = scenegen.tiny_scene(seed=4, n_pts=40, n_grid=4, t_hi=3, with_stats=False)
    uv = orc.observations(s)
    S = _dense_rcs(s, uv, 1e-3)
    n = s.n_cams
    nz = np.array([[np.abs(S[9 * i:9 * i + 9, 9 * j:9 * j + 9]).max() > 0 for j in range(n)] for i in range(n)])
    assert nz.sum() < n * n           # a sparse case: some cameras share no point
    alpha = nz.sum() / n ** 2
    P = orc.Problem.from_scene(s, uv)
    assert P.n_rows == n
    for c in (9, 11):
        YB = (alpha * n * n + n) / 2 * c * c * 8 + (alpha * n * n + n) / 2 * 3 * 4 + n * 4
        assert abs(P.bsmc_bytes(c) - YB) < 1e-6 * YB
        YC = alpha * n * n * c * c * 8 + alpha * n * n * c * c * 4 + n * c * 4
        ratio10 = (6 * alpha * n * c * c + 2 * c) / (2 * alpha * n * c * c + 2 * c * c + 3 * alpha * n + 5)
        assert abs(YC / YB - ratio10) < 1e-12 * ratio10


def test_invalid_inputs_rejected():
    s = small_scene(seed=1)
    uv = orc.observations(s)
    bad = s.obs_cam.copy(); bad[3] = s.n_cams
    with pytest.raises(ValueError):
        orc.Problem(s.n_cams, s.n_pts, bad, s.obs_pt, uv)
    # duplicate (camera, point) observation
    oc = np.concatenate([s.obs_cam, s.obs_cam[:1]]); op = np.concatenate([s.obs_pt, s.obs_pt[:1]])
    with pytest.raises(ValueError):
        orc.Problem(s.n_cams, s.n_pts, oc, op, np.concatenate([uv, uv[:, :1]], axis=1))
