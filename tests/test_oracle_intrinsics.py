"""Pins of the shared-intrinsics reference (6 exterior unknowns per image, 5
interior per physical camera; Sec. 4.1 counts c = 11, Table 2 lists fewer
cameras than images):
  - its Jacobian blocks against central finite differences;
  - its point-by-point RCS against dense elimination of the points from the
    full damped normal matrix (LAPACK);
  - with one physical camera per image and the principal point at 0 the
    model is the 9-parameter one, so the RCS entries of (w, t, f, k1, k2)
    equal the C oracle's (an independent implementation);
  - symmetry, positive definiteness with damping, and the block pattern
    against the non-zero blocks of the dense RCS."""
import numpy as np
import pytest

from oracle import intrinsics as I
from oracle import oracle as orc
from paper_2307_08383_amd import scenegen


def _scene(n_phys=3, n_pts=300, nx=4, ny=3, seed=5):
    return scenegen.shared_intrinsics_scene(seed=seed, nx=nx, ny=ny, n_pts=n_pts, n_phys=n_phys)


def _uv(s):
    pu, pv = I.project(s.ext_true, s.intr_true, s.img_cam, s.pts_true, s.obs_img, s.obs_pt)
    return np.stack([pu.v, pv.v]) + s.noise


def test_jacobians_finite_differences():
    s = _scene(n_pts=60)
    uv = _uv(s)
    F, e, Je, Jq, Jp = I.linearize(s.ext_init, s.intr_init, s.img_cam, s.pts_init, s.obs_img, s.obs_pt, uv)

    def resid(ext, intr, pts):
        pu, pv = I.project(ext, intr, s.img_cam, pts, s.obs_img, s.obs_pt)
        return np.stack([pu.v - uv[0], pv.v - uv[1]], axis=1)

    for k in range(len(s.obs_img)):
        i, p = s.obs_img[k], s.obs_pt[k]
        c = s.img_cam[i]
        for blockname, arr, row, J, n in (("ext", s.ext_init, i, Je, 6), ("intr", s.intr_init, c, Jq, 5),
                                          ("pt", s.pts_init, p, Jp, 3)):
            for j in range(n):
                h = 1e-6 * max(1.0, abs(arr[row, j]))
                plus, minus = arr.copy(), arr.copy()
                plus[row, j] += h
                minus[row, j] -= h
                args_p = {"ext": (plus, s.intr_init, s.pts_init), "intr": (s.ext_init, plus, s.pts_init),
                          "pt": (s.ext_init, s.intr_init, plus)}[blockname]
                args_m = {"ext": (minus, s.intr_init, s.pts_init), "intr": (s.ext_init, minus, s.pts_init),
                          "pt": (s.ext_init, s.intr_init, minus)}[blockname]
                fd = (resid(*args_p)[k] - resid(*args_m)[k]) / (2 * h)
                scale = max(1.0, np.abs(J[k]).max())
                assert np.abs(fd - J[k][:, j]).max() <= 1e-6 * scale, (blockname, k, j)
        if k > 40:
            break


@pytest.mark.parametrize("n_phys,fixed", [(3, False), (1, False), (3, True)])
def test_rcs_equals_dense_elimination(n_phys, fixed):
    s = _scene(n_phys=n_phys, n_pts=150)
    if fixed:
        s.img_fixed[[0, 5]] = 1
    uv = _uv(s)
    P = I.SharedProblem(s.n_img, s.n_phys, s.img_cam, s.n_pts, s.obs_img, s.obs_pt, uv, s.img_fixed)
    lam = 1e-3
    S, b, F = P.rcs(s.ext_init, s.intr_init, s.pts_init, lam)
    # dense: full Jacobian over [camera-side unknowns, points], H = J^T J + lam diag
    _, e, Je, Jq, Jp = I.linearize(s.ext_init, s.intr_init, s.img_cam, s.pts_init, s.obs_img, s.obs_pt, uv)
    m = P.m
    J = np.zeros((2 * s.n_obs, m + 3 * s.n_pts))
    for k in range(s.n_obs):
        i, p = s.obs_img[k], s.obs_pt[k]
        if P.img_row[i] >= 0:
            J[2 * k:2 * k + 2, P.ext_index(i)] = Je[k]
        J[2 * k:2 * k + 2, P.intr_index(s.img_cam[i])] = Jq[k]
        J[2 * k:2 * k + 2, m + 3 * p:m + 3 * p + 3] = Jp[k]
    H = J.T @ J
    H[np.diag_indices_from(H)] *= 1.0 + lam
    g = -J.T @ e.ravel()
    S_ref = H[:m, :m] - H[:m, m:] @ np.linalg.solve(H[m:, m:], H[m:, :m])
    b_ref = g[:m] - H[:m, m:] @ np.linalg.solve(H[m:, m:], g[m:])
    assert np.abs(S - S_ref).max() <= 1e-10 * np.abs(S_ref).max()
    assert np.abs(b - b_ref).max() <= 1e-10 * np.abs(b_ref).max()
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    assert np.linalg.eigvalsh(S).min() > 0


def test_one_camera_per_image_is_the_nine_parameter_model():
    s = _scene(n_phys=12, n_pts=200)          # 4 x 3 = 12 images, camera i takes image i
    s.intr_true[:, 1:3] = 0.0                 # principal point at the origin
    s.intr_init[:, 1:3] = 0.0
    uv = _uv(s)
    P = I.SharedProblem(s.n_img, s.n_phys, s.img_cam, s.n_pts, s.obs_img, s.obs_pt, uv)
    S, b, F = P.rcs(s.ext_init, s.intr_init, s.pts_init, 1e-3)
    cams9 = np.concatenate([s.ext_init, s.intr_init[:, [0, 3, 4]]], axis=1)
    O = orc.Problem(s.n_img, s.n_pts, s.obs_img, s.obs_pt, uv)
    F9 = O.linearize(cams9, s.pts_init)
    O.form_rcs(1e-3)
    blk9, rhs9 = O.rcs()
    rp9, ci9 = O.pattern()
    assert abs(F - F9) <= 1e-12 * F9
    idx = lambda i: np.concatenate([P.ext_index(i), P.intr_index(i)[[0, 3, 4]]])
    for r in range(s.n_img):
        for k in range(rp9[r], rp9[r + 1]):
            c = ci9[k]
            ref = blk9[k]
            got = S[np.ix_(idx(r), idx(c))]
            assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
        assert np.abs(b[idx(r)] - rhs9[r]).max() <= 1e-9 * np.abs(rhs9[r]).max()


def test_pattern_and_padded_blocks():
    s = _scene(n_phys=2, n_pts=120, nx=5, ny=4)
    uv = _uv(s)
    P = I.SharedProblem(s.n_img, s.n_phys, s.img_cam, s.n_pts, s.obs_img, s.obs_pt, uv)
    S, b, _ = P.rcs(s.ext_init, s.intr_init, s.pts_init, 1e-3)
    rp, ci, blk, rhs = P.padded_blocks(S, b)
    node, slot = P.nodes_of_unknowns()
    n_nodes = len(rp) - 1
    nz = np.zeros((n_nodes, n_nodes), bool)
    for x in range(P.m):
        for y in range(P.m):
            if S[x, y] != 0.0:
                nz[node[x], node[y]] = True
    present = np.zeros((n_nodes, n_nodes), bool)
    for u in range(n_nodes):
        present[u, ci[rp[u]:rp[u + 1]]] = True
        assert ci[rp[u]] == u and np.all(np.diff(ci[rp[u]:rp[u + 1]]) > 0)
    assert np.array_equal(present, np.triu(nz))
    assert nz[:P.n_free, P.n_free:].all()   # every image couples with every camera here
    for u in range(n_nodes):
        nreal = 6 if u < P.n_free else 5
        d = blk[rp[u]]
        assert np.array_equal(d[nreal:, nreal:], np.eye(9 - nreal))
        assert not d[nreal:, :nreal].any() and not rhs[u, nreal:].any()


def test_dense_step_matches_reduced_system_and_lm_converges():
    """The step over all unknowns (dense solve of Eq. (1)) has the camera
    part that solves the reduced system of Eq. (4), and the LM reference
    with it reaches the noise floor: F close to (2 n_obs - n_unknowns) s^2 / 2."""
    s = _scene(n_phys=3, n_pts=300)
    uv = _uv(s)
    P = I.SharedProblem(s.n_img, s.n_phys, s.img_cam, s.n_pts, s.obs_img, s.obs_pt, uv)
    S, b, F = P.rcs(s.ext_init, s.intr_init, s.pts_init, 1e-4)
    dx = np.linalg.solve(S, b)
    de, dq, dp, F2, pred = P.dense_step(s.ext_init, s.intr_init, s.pts_init, 1e-4)
    assert F2 == F
    assert np.abs(dx[:6 * s.n_img].reshape(-1, 6) - de).max() <= 1e-9 * np.abs(de).max()
    assert np.abs(dx[6 * s.n_img:].reshape(-1, 5) - dq).max() <= 1e-9 * np.abs(dq).max()
    _, _, _, hist = I.lm_run(P, s.ext_init, s.intr_init, s.pts_init, 8)
    dof = 2 * s.n_obs - (6 * s.n_img + 5 * s.n_phys + 3 * s.n_pts - 7)
    F_end = hist[-1]["cost_new"] if hist[-1]["accepted"] else hist[-1]["cost"]
    assert 0.5 * dof * 0.25 * 0.7 < F_end < 0.5 * dof * 0.25 * 1.3
