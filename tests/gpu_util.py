"""Helpers shared by the GPU tests: run a scene through the HIP library and
through the oracle on identical inputs."""
import numpy as np

from oracle import oracle as orc


def torch_dev():
    import torch
    return torch.device("cuda:0")


def T(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=torch_dev())


def create(scene, uv, precision=0, cam_fixed=None):
    import torch
    from paper_2307_08383_amd import ba
    cf = cam_fixed if cam_fixed is not None else (scene.cam_fixed if scene.cam_fixed.any() else None)
    return ba.ba_create(scene.n_cams, scene.n_pts, T(scene.obs_cam, torch.int32), T(scene.obs_pt, torch.int32),
                        T(uv, torch.float64), None if cf is None else T(cf, torch.uint8), precision=precision)


def block_errors(blk, ref, rp, ci):
    """Per-block error ||dS||_F / max(||S||_F, 1e-3 sqrt(||S_ii||_F ||S_jj||_F)),
    the floor guarding blocks that nearly cancel in the Schur complement."""
    n = len(rp) - 1
    dn = np.array([np.linalg.norm(ref[rp[r]]) for r in range(n)])
    errs = np.empty(len(ci))
    raw = np.empty(len(ci))
    for r in range(n):
        for k in range(rp[r], rp[r + 1]):
            c = ci[k]
            nd = np.linalg.norm(blk[k] - ref[k])
            nr = np.linalg.norm(ref[k])
            errs[k] = nd / max(nr, 1e-3 * np.sqrt(dn[r] * dn[c]))
            raw[k] = nd / nr if nr > 0 else (0.0 if nd == 0 else np.inf)
    return errs, raw


def check_against_oracle(ctx, P, cams, pts, lam, precision, rng):
    """J, e, RCS and the point terms (through back-substitution) of ctx
    against the oracle at (cams, pts, lam): J to 1e-11 (FP64) / 1e-6 (FP32
    records) of each row's scale, blocks 1e-10 / 1e-4 in the floored
    metric, rhs 1e-9 / 1e-4, dx_p 1e-10 / 1e-4 of its largest entry."""
    import torch
    from paper_2307_08383_amd import ba
    F_ref = P.linearize(cams, pts)
    P.form_rcs(lam)
    e_ref, Jc, Jp = P.linearization()
    J, e = ba.ba_get_jacobians(ctx)
    J_ref = np.concatenate([Jc.reshape(-1, 18), Jp.reshape(-1, 6)], axis=1)
    scale = np.abs(J_ref).max(axis=1, keepdims=True)
    jtol = 1e-11 if precision == 0 else 1e-6
    assert (np.abs(J - J_ref) / scale).max() <= jtol
    np.testing.assert_allclose(e, e_ref, rtol=0, atol=1e-9)
    blk, rhs = ba.ba_get_rcs(ctx)
    blk_ref, rhs_ref = P.rcs()
    rp, ci = P.pattern()
    errs, raw = block_errors(blk, blk_ref, rp, ci)
    assert errs.max() <= (1e-10 if precision == 0 else 1e-4), (errs.max(), raw.max())
    rerr = np.linalg.norm(rhs - rhs_ref, axis=1) / np.linalg.norm(rhs_ref, axis=1)
    assert rerr.max() <= (1e-9 if precision == 0 else 1e-4), rerr.max()
    # back-substitution reads the point terms (Cholesky factor of V*, L^-1 l_p)
    # that the fused kernel stored
    dxc = rng.standard_normal((P.n_rows, 9)) * 1e-3
    dxp = torch.empty((P.n_pts, 3), dtype=torch.float64, device="cuda")
    ba.ba_back_substitute(ctx, T(dxc, torch.float64), dxp)
    dxp_ref = P.back_substitute(dxc)
    btol = 1e-10 if precision == 0 else 1e-4
    assert np.abs(dxp.cpu().numpy() - dxp_ref).max() <= btol * np.abs(dxp_ref).max()
    return F_ref, J, e, blk, rhs
