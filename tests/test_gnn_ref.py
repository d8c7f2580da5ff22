"""Pins of the CPU reference of the learned block-Jacobi correction."""
import numpy as np
import pytest

from oracle import gnn_ref as G
from oracle import oracle as orc
from paper_2307_08383_amd import scenegen


@pytest.fixture(scope="module")
def feat():
    s = scenegen.tiny_scene(seed=3, n_pts=200, with_stats=False)
    P = orc.Problem.from_scene(s)
    P.linearize(s.cams_init, s.pts_init)
    P.form_rcs(1e-3)
    rp, ci = P.pattern()
    blk, _ = P.rcs()
    return G.features(rp, ci, blk), (rp, ci, blk)


def _probes(n, k=4, seed=0):
    rng = np.random.default_rng(seed)
    return rng.choice([-1.0, 1.0], size=(k, n, 9))


def test_normalised_blocks(feat):
    f, (rp, ci, blk) = feat
    # A = L^-1 S L^-T has identity diagonal blocks; check one edge and the
    # symmetric twin relation A_ji = A_ij^T
    g = f["graph"]
    e = 5
    i, j = g["src"][e], g["dst"][e]
    Sij = blk[g["blk"][e]] if g["tr"][e] == 0 else blk[g["blk"][e]].T
    np.testing.assert_allclose(f["L"][i] @ f["A"][e] @ f["L"][j].T, Sij, rtol=1e-10, atol=1e-10 * np.abs(Sij).max())
    np.testing.assert_allclose(f["A"][g["twin"][e]], f["A"][e].T, atol=1e-12)
    # A is the congruence of S: its dense form has unit diagonal blocks and
    # the same eigenvalues as M^-1 S with M = blockdiag(S_ii)
    n = g["n"]
    Ad = np.zeros((9 * n, 9 * n))
    for ii in range(n):
        Ad[9 * ii:9 * ii + 9, 9 * ii:9 * ii + 9] = np.eye(9)
    for e in range(len(g["src"])):
        a, b = g["src"][e], g["dst"][e]
        Ad[9 * a:9 * a + 9, 9 * b:9 * b + 9] = f["A"][e]
    S = np.zeros_like(Ad)
    for r in range(n):
        for k in range(rp[r], rp[r + 1]):
            c = ci[k]
            S[9 * r:9 * r + 9, 9 * c:9 * c + 9] = blk[k]
            S[9 * c:9 * c + 9, 9 * r:9 * r + 9] = blk[k].T
    M = np.zeros_like(S)
    for r in range(n):
        M[9 * r:9 * r + 9, 9 * r:9 * r + 9] = S[9 * r:9 * r + 9, 9 * r:9 * r + 9]
    ev1 = np.sort(np.linalg.eigvalsh(Ad))
    ev2 = np.sort(np.real(np.linalg.eigvals(np.linalg.solve(M, S))))
    np.testing.assert_allclose(ev1, ev2, rtol=1e-8, atol=1e-10)


def test_zero_decoder_is_block_jacobi(feat):
    f, (rp, ci, blk) = feat
    w = G.init_params(seed=1, zero_decoder=True)
    o, _ = G.forward(w, f)
    assert np.all(o == 0.0)
    Pm = G.preconditioner(o, f["L"])
    for i in range(len(rp) - 1):
        np.testing.assert_allclose(Pm[i], np.linalg.inv(blk[rp[i]]), rtol=1e-9, atol=1e-12 * np.abs(Pm[i]).max())


def test_preconditioner_blocks_are_spd(feat):
    f, _ = feat
    rng = np.random.default_rng(2)
    o = rng.normal(0, 1.0, size=(f["graph"]["n"], G.F_OUT))
    Pm = G.preconditioner(o, f["L"])
    for Pi in Pm:
        assert np.allclose(Pi, Pi.T, atol=1e-12 * np.abs(Pi).max())
        assert np.linalg.eigvalsh(Pi).min() > 0


def test_output_gradient_finite_differences(feat):
    f, _ = feat
    n = f["graph"]["n"]
    z = _probes(n)
    y = np.stack([G.normalised_product(f, zp) for zp in z])
    rng = np.random.default_rng(3)
    o = rng.normal(0, 0.1, size=(n, G.F_OUT))
    loss, do = G.loss_and_dout(o, z, y)
    for _ in range(30):
        i, c = rng.integers(n), rng.integers(45)
        h = 1e-6
        op = o.copy(); op[i, c] += h
        om = o.copy(); om[i, c] -= h
        fd = (G.loss_and_dout(op, z, y)[0] - G.loss_and_dout(om, z, y)[0]) / (2 * h)
        assert abs(fd - do[i, c]) <= 1e-6 * max(1.0, np.abs(do).max())


def test_parameter_gradient_finite_differences(feat):
    f, _ = feat
    n = f["graph"]["n"]
    z = _probes(n, k=2)
    w = G.init_params(seed=4, zero_decoder=False)
    loss, grad, _ = G.loss_and_grad(w, f, z)
    rng = np.random.default_rng(5)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in G.PARAM_SHAPES])
    gscale = np.abs(grad).max()
    checked = 0
    for t, (name, shape) in enumerate(G.PARAM_SHAPES):
        for _ in range(3):
            k = offs[t] + rng.integers(offs[t + 1] - offs[t])
            h = 1e-6 * max(1.0, abs(w[k]))
            wp = w.copy(); wp[k] += h
            wm = w.copy(); wm[k] -= h
            fd = (G.loss_and_grad(wp, f, z)[0] - G.loss_and_grad(wm, f, z)[0]) / (2 * h)
            assert abs(fd - grad[k]) <= 1e-6 * gscale + 1e-5 * abs(fd), (name, fd, grad[k])
            checked += 1
    assert checked == 3 * len(G.PARAM_SHAPES)


def test_hutchinson_estimates_frobenius(feat):
    """E_z |(B A - I) z|^2 = ||B A - I||_F^2 for Rademacher z."""
    f, _ = feat
    n = f["graph"]["n"]
    rng = np.random.default_rng(6)
    o = rng.normal(0, 0.05, size=(n, G.F_OUT))
    z = rng.choice([-1.0, 1.0], size=(600, n, 9))
    y = np.stack([G.normalised_product(f, zp) for zp in z])
    est, _ = G.loss_and_dout(o, z, y)
    # exact ||B A - I||_F^2 / (9 n) from dense columns
    Lt = G.factor_from_output(o)
    B = Lt @ np.transpose(Lt, (0, 2, 1))
    tot = 0.0
    for col in range(9 * n):
        e = np.zeros((n, 9)); e.flat[col] = 1.0
        r = np.einsum("nij,nj->ni", B, G.normalised_product(f, e)) - e
        tot += (r * r).sum()
    exact = tot / (9 * n)
    assert abs(est - exact) <= 0.05 * exact


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 0.0])
    r = G.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7 and r[4] == 0.0
    assert abs(r[3] + 3.14159) < 2 ** -7 * 4


# ---------------------------------------------------------------------------
# factorised head
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def grid_feat():
    from oracle import fsai
    s = scenegen.aerial_grid_scene(seed=9, nx=5, ny=4, n_pts=1500, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    P.linearize(s.cams_init, s.pts_init)
    P.form_rcs(1e-3)
    rp, ci = P.pattern()
    blk, _ = P.rcs()
    cnt = fsai.shared_points(P.n_rows, P.cam_row(), s.obs_cam, s.obs_pt)
    J = fsai.lower_sets(rp, ci, cnt, 3)
    return G.features(rp, ci, blk), J, (rp, ci, blk, cnt)


def test_zero_head_is_block_jacobi(grid_feat):
    f, J, (rp, ci, blk, cnt) = grid_feat
    w = G.init_params(0, zero_decoder=True)
    rows, _ = G.fsai_factor(w, f, J)
    for Gi in rows:
        np.testing.assert_array_equal(Gi[:-1], 0.0)
        np.testing.assert_array_equal(Gi[-1], np.eye(9))
    loss, _ = G.kaporin_loss(rows, f, J)
    assert abs(loss - 1.0) <= 1e-12          # tr(I) per row, log det 0
    Gorig = G.fsai_preconditioner_factor(rows, J, f["L"])
    for i, Gi in enumerate(Gorig):
        np.testing.assert_allclose(Gi[-1], np.linalg.inv(f["L"][i]), rtol=1e-12, atol=1e-15)


def test_kaporin_stationary_at_exact_fsai(grid_feat):
    # the oracle's FSAI factor (pinned separately), mapped to normalised
    # coordinates, is a stationary point of the reference's Kaporin loss
    from oracle import fsai
    f, J, (rp, ci, blk, cnt) = grid_feat
    Gd, _, Jo = fsai.fsai(blk, rp, ci, cnt, cap=3)
    assert Jo == J
    rows = []
    for i, Ji in enumerate(J):
        rows.append(np.stack([Gd[9 * i:9 * i + 9, 9 * j:9 * j + 9] @ f["L"][j] for j in Ji]))
    loss, grads = G.kaporin_loss(rows, f, J)
    for Gi, dGi in zip(rows, grads):
        # lower-triangular part of the diagonal block and the off-diagonal blocks
        mask = np.ones_like(dGi)
        mask[-1] = np.tril(np.ones((9, 9)))
        assert np.abs(dGi * mask).max() <= 1e-9 * max(1.0, np.abs(Gi).max())
    assert loss < 1.0
    # and below any perturbation of it
    rng = np.random.default_rng(1)
    for _ in range(3):
        pert = [Gi + 1e-3 * rng.normal(size=Gi.shape) * np.concatenate(
            [np.ones((len(Gi) - 1, 9, 9)), np.tril(np.ones((1, 9, 9)))]) for Gi in rows]
        assert G.kaporin_loss(pert, f, J)[0] > loss


def test_fsai_head_gradient_finite_differences(grid_feat):
    f, J, _ = grid_feat
    w = G.init_params(2, zero_decoder=False, decoder_scale=0.2)
    d = G.unflatten(w.copy())
    d["ao"][:] = 0.3
    d["bo2"][:] = np.random.default_rng(3).normal(0, 0.02, size=d["bo2"].shape)
    d["bo1"][:] = np.random.default_rng(4).normal(0, 0.05, size=d["bo1"].shape)
    w = G.flatten(d)
    loss, grad = G.fsai_loss_and_grad(w, f, J)
    rng = np.random.default_rng(4)
    names = {name: (o, int(np.prod(shape))) for name, shape, o in
             [(n_, s_, o_) for (n_, s_), o_ in zip(G.PARAM_SHAPES, np.cumsum([0] + [int(np.prod(s)) for _, s in G.PARAM_SHAPES])[:-1])]}
    for name in ["Wo1", "bo1", "Wo2", "bo2", "ao", "Wd", "bd", "M2", "U0", "We", "Wn"]:
        off, size = names[name]
        for k in rng.choice(size, size=3, replace=False):
            idx = off + int(k)
            h = 1e-6 * max(1.0, abs(w[idx]))
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            lp = G.kaporin_loss(G.fsai_factor(wp, f, J)[0], f, J)[0]
            lm = G.kaporin_loss(G.fsai_factor(wm, f, J)[0], f, J)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[idx]) <= 1e-6 * np.abs(grad).max() + 1e-5 * abs(fd), (name, k, fd, grad[idx])


def test_first_order_skip_improves_on_block_jacobi(grid_feat):
    # ao = 1 gives Ghat_ij = -A_ij, the first-order approximation of the
    # inverse factor: lower Kaporin functional than block-Jacobi
    f, J, _ = grid_feat
    d = G.unflatten(G.init_params(0, zero_decoder=True))
    d["ao"][:81] = 1.0
    rows, _ = G.fsai_factor(G.flatten(d), f, J)
    assert G.kaporin_loss(rows, f, J)[0] < 1.0
