"""A learned preconditioner that fails falls back to block-Jacobi (needs a GPU).

The network's diagonal factor entries are exp(.) of its decoder output; with
a decoder bias of 1e4 they overflow to +inf in FP32, so the preconditioner
is not finite and the first d^T S d of PCG is NaN (treated as "not
positive").  Both the block head (LEARNED) and the factorised head
(LEARNED_FSAI) must then solve with block-Jacobi (Sec. 3.2's block-diagonal
preconditioner) in the same call and report it; the LM step is accepted and
equals a plain block-Jacobi step bit for bit.  Nothing here makes the GPU
fault: the overflow only produces non-finite values."""
import numpy as np
import pytest

from oracle import gnn_ref
from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from gpu_util import T, create

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")


def _overflowing_params():
    d = gnn_ref.unflatten(gnn_ref.init_params(0).copy())
    d["bd"][:9] = 1e4    # diagonal of every Lt_i: exp(1e4) = inf in FP32
    return gnn_ref.flatten(d).astype(np.float32)


@pytest.mark.parametrize("pre", ["learned", "learned_fsai"])
def test_failed_learned_preconditioner_falls_back(pre):
    code = ba.BA_PRECOND_LEARNED if pre == "learned" else ba.BA_PRECOND_LEARNED_FSAI
    s = scenegen.tiny_scene(seed=0, with_stats=False)
    uv = orc.observations(s)
    ctx = create(s, uv)
    ref = create(s, uv)
    net = ba.ba_gnn_create(_overflowing_params())
    try:
        ba.ba_set_preconditioner_net(ctx, net)
        cams = T(s.cams_init, torch.float64)
        pts = T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        info = ba.ba_lm_step(ctx, cams, pts, st, precond=code)
        cams_r = T(s.cams_init, torch.float64)
        pts_r = T(s.pts_init, torch.float64)
        st_r = ba.new_lm_state(1e-4)
        info_r = ba.ba_lm_step(ref, cams_r, pts_r, st_r)
        assert info["precond_fallback"] == 1 and info_r["precond_fallback"] == 0
        assert info["accepted"] == 1 and info["pcg_status"] == ba.BA_OK
        assert info["pcg_iters"] == info_r["pcg_iters"]
        assert info["cost_new"] == info_r["cost_new"] and st.lam == st_r.lam
        assert torch.equal(cams, cams_r) and torch.equal(pts, pts_r)
        # the same through ba_pcg_solve on the next RCS
        ba.ba_linearize(ctx, cams, pts)
        ba.ba_form_rcs(ctx, st.lam)
        ba.ba_linearize(ref, cams_r, pts_r)
        ba.ba_form_rcs(ref, st_r.lam)
        n_rows = ba.ba_get_sizes(ctx)["n_rows"]
        x = torch.empty((n_rows, 9), dtype=torch.float64, device="cuda")
        x_r = torch.empty_like(x)
        sol = ba.ba_pcg_solve(ctx, x, tol=1e-8, precond=code)
        sol_r = ba.ba_pcg_solve(ref, x_r, tol=1e-8)
        assert sol["precond_fallback"] == 1 and sol["status"] == ba.BA_OK
        assert sol["iters"] == sol_r["iters"] and torch.equal(x, x_r)
    finally:
        ba.ba_set_preconditioner_net(ctx, None)
        ba.ba_gnn_destroy(net)
        ba.ba_destroy(ctx)
        ba.ba_destroy(ref)
