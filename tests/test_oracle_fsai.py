"""Pins of the oracle's FSAI preconditioner against facts that do not depend
on it: the block-Jacobi and full-pattern special cases (textbook Cholesky
inverses), the defining conditions on a truncated pattern, the minimality
of the Kaporin functional, brute-force common-point counts, and the PCG
solution against a dense solve."""
import numpy as np
import pytest

from oracle import fsai
from oracle import oracle as orc
from paper_2307_08383_amd import scenegen


def _rcs(scene, lam=1e-3, obs=None):
    oc, op = (scene.obs_cam, scene.obs_pt) if obs is None else obs
    uv = orc.project(scene.cams_true, scene.pts_true, oc, op)
    P = orc.Problem(scene.n_cams, scene.n_pts, oc, op, uv)
    P.linearize(scene.cams_init, scene.pts_init)
    P.form_rcs(lam)
    blk, rhs = P.rcs()
    rp, ci = P.pattern()
    cnt = fsai.shared_points(P.n_rows, P.cam_row(), oc, op)
    return P, blk, rhs, rp, ci, cnt


@pytest.fixture(scope="module")
def grid_case():
    # 5 x 4 cameras: a banded pattern where rows have several lower neighbours
    s = scenegen.aerial_grid_scene(seed=9, nx=5, ny=4, n_pts=1500, with_stats=False)
    return s, _rcs(s)


def test_shared_points_brute_force(grid_case):
    s, (P, blk, rhs, rp, ci, cnt) = grid_case
    cr = P.cam_row()
    sets = [set() for _ in range(P.n_rows)]
    for c, p in zip(s.obs_cam, s.obs_pt):
        sets[cr[c]].add(int(p))
    for r in range(P.n_rows):
        for k in range(rp[r] + 1, rp[r + 1]):
            assert cnt[(r, int(ci[k]))] == len(sets[r] & sets[int(ci[k])]) > 0
    pairs = {(r, int(ci[k])) for r in range(P.n_rows) for k in range(rp[r] + 1, rp[r + 1])}
    assert set(cnt) == pairs


def test_block_diagonal_case_is_block_jacobi(grid_case):
    s, (P, blk, rhs, rp, ci, cnt) = grid_case
    b2 = blk.copy()
    diag = set(int(k) for k in rp[:-1])
    for k in range(len(b2)):
        if k not in diag:
            b2[k] = 0.0
    G, Gs, J = fsai.fsai(b2, rp, ci, cnt, cap=100)
    for r in range(P.n_rows):
        Linv = np.linalg.inv(np.linalg.cholesky(blk[rp[r]]))
        np.testing.assert_allclose(Gs[rp[r]], Linv, rtol=0, atol=1e-12 * np.abs(Linv).max())
    off = [k for k in range(len(Gs)) if k not in diag]
    assert np.abs(Gs[off]).max() <= 1e-12 * np.abs(Gs).max()


def test_full_pattern_is_inverse_cholesky_factor():
    s = scenegen.tiny_scene(seed=2, n_pts=40, with_stats=False)
    n_c = 5
    oc = np.repeat(np.arange(n_c, dtype=np.int32)[None, :], 40, axis=0).ravel()
    op = np.repeat(np.arange(40, dtype=np.int32), n_c)
    sub = scenegen.Scene(**{**s.__dict__})
    sub.n_cams = n_c
    sub.cams_true, sub.cams_init = s.cams_true[:n_c], s.cams_init[:n_c]
    P, blk, rhs, rp, ci, cnt = _rcs(sub, obs=(oc, op))
    assert len(ci) == n_c * (n_c + 1) // 2          # every pair co-observes
    S = fsai.dense_rcs(blk, rp, ci)
    G, Gs, J = fsai.fsai(blk, rp, ci, cnt, cap=100)
    G_ref = np.linalg.inv(np.linalg.cholesky(S))      # textbook S^-1 = L^-T L^-1
    np.testing.assert_allclose(G, G_ref, rtol=0, atol=1e-10 * np.abs(G_ref).max())
    b = rhs.ravel()
    x, it, rel = fsai.pcg(lambda v: S @ v, b, lambda v: G.T @ (G @ v), tol=1e-12)
    assert it == 1 and rel <= 1e-12


@pytest.mark.parametrize("cap", [1, 2, 100])
def test_defining_conditions(grid_case, cap):
    s, (P, blk, rhs, rp, ci, cnt) = grid_case
    S = fsai.dense_rcs(blk, rp, ci)
    G, Gs, J = fsai.fsai(blk, rp, ci, cnt, cap=cap)
    n = P.n_rows
    GS = G @ S
    GSG = GS @ G.T
    scale = np.abs(S).max() * np.abs(G).max()
    truncated = False
    for i in range(n):
        n_low = sum(1 for r in range(n) for k in range(rp[r] + 1, rp[r + 1]) if ci[k] == i)
        truncated |= n_low > cap
        for j in range(n):
            blkG = G[9 * i:9 * i + 9, 9 * j:9 * j + 9]
            if j not in J[i]:
                assert not blkG.any()
            elif j != i:
                assert np.abs(GS[9 * i:9 * i + 9, 9 * j:9 * j + 9]).max() <= 1e-10 * scale
        np.testing.assert_allclose(GSG[9 * i:9 * i + 9, 9 * i:9 * i + 9], np.eye(9), rtol=0, atol=1e-10)
        Gii = G[9 * i:9 * i + 9, 9 * i:9 * i + 9]
        # lower triangular up to rounding (C^T D = C^-1 in exact arithmetic)
        assert np.abs(np.triu(Gii, 1)).max() <= 1e-12 * np.abs(Gii).max() and np.all(np.diag(Gii) > 0)
    if cap < 100:
        assert truncated
    # truncation keeps the neighbours with the most common points
    for i in range(n):
        low = [r for r in range(n) for k in range(rp[r] + 1, rp[r + 1]) if ci[k] == i]
        kept = set(J[i][:-1])
        for a in kept:
            for b in set(low) - kept:
                assert cnt[(a, i)] > cnt[(b, i)] or (cnt[(a, i)] == cnt[(b, i)] and a < b)


def test_kaporin_minimum(grid_case):
    s, (P, blk, rhs, rp, ci, cnt) = grid_case
    S = fsai.dense_rcs(blk, rp, ci)
    G, Gs, J = fsai.fsai(blk, rp, ci, cnt, cap=2)
    f0 = fsai.kaporin(G, S)
    mask = np.zeros_like(G, dtype=bool)
    for i, Ji in enumerate(J):
        for j in Ji:
            m = np.ones((9, 9), bool) if j != i else np.tril(np.ones((9, 9), bool))
            mask[9 * i:9 * i + 9, 9 * j:9 * j + 9] = m
    # perturbations D = Dhat L^-1 with Dhat O(1) in the block-Jacobi-normalised
    # coordinates (G_ii L_i is O(1) there); D keeps the pattern and the
    # lower-triangular diagonal blocks
    Linv = np.zeros_like(G)
    for i in range(P.n_rows):
        Linv[9 * i:9 * i + 9, 9 * i:9 * i + 9] = np.linalg.inv(np.linalg.cholesky(S[9 * i:9 * i + 9, 9 * i:9 * i + 9]))
    rng = np.random.default_rng(0)
    for _ in range(4):
        D = (rng.normal(size=G.shape) * mask) @ Linv
        eps = 1e-4
        fp, fm = fsai.kaporin(G + eps * D, S), fsai.kaporin(G - eps * D, S)
        assert fp > f0 and fm > f0
        # stationary: the odd part of f along D (eps |grad.D|) is far below
        # the even part (eps^2 D^T f'' D / 2); at block-Jacobi it is not
        assert abs(fp - fm) <= 1e-2 * (fp + fm - 2 * f0)
        gp, gm = fsai.kaporin(Linv + eps * D, S), fsai.kaporin(Linv - eps * D, S)
        assert abs(gp - gm) > abs(gp + gm - 2 * fsai.kaporin(Linv, S))
    # block-Jacobi (G_ii = L_i^-1, nothing else) has the larger functional
    assert fsai.kaporin(Linv, S) > f0


def test_pcg_solution_against_dense_solve(grid_case):
    s, (P, blk, rhs, rp, ci, cnt) = grid_case
    S = fsai.dense_rcs(blk, rp, ci)
    b = rhs.ravel()
    G, Gs, J = fsai.fsai(blk, rp, ci, cnt, cap=3)
    x, it, rel = fsai.pcg(lambda v: S @ v, b, lambda v: G.T @ (G @ v), tol=1e-13, max_iter=2000)
    x_ref = np.linalg.solve(S, b)
    assert rel <= 1e-13
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-8 * np.abs(x_ref).max())
    # the numpy recurrence with block-Jacobi matches the C oracle's count
    Minv = np.zeros_like(S)
    for i in range(P.n_rows):
        Minv[9 * i:9 * i + 9, 9 * i:9 * i + 9] = np.linalg.inv(S[9 * i:9 * i + 9, 9 * i:9 * i + 9])
    _, it_bj, _ = fsai.pcg(lambda v: S @ v, b, lambda v: Minv @ v, tol=1e-8, max_iter=2000)
    _, oinfo = P.pcg(tol=1e-8, max_iter=2000)
    assert abs(it_bj - oinfo["iters"]) <= 1
    # slots round trip
    np.testing.assert_array_equal(fsai.dense_from_slots(Gs, rp, ci), G)
