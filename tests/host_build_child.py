"""Child process of test_gpu_host_build.py: builds contexts on the scenes
named on the command line with the thread count BA_THREADS from the
environment and prints a JSON line of hashes (pattern, RCS, a few PCG
iterations with block-Jacobi, FSAI and the learned factor, one LM step)."""
import hashlib
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import numpy as np  # noqa: E402
import torch  # noqa: E402

from oracle import intrinsics as I  # noqa: E402
from oracle import oracle as orc  # noqa: E402
from paper_2307_08383_amd import ba, learned_precond as lp, scenegen  # noqa: E402

dev = torch.device("cuda:0")


def T(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)


def digest(*arrs):
    return hashlib.sha256(b"".join(np.ascontiguousarray(a).tobytes() for a in arrs)).hexdigest()


def nine(s):
    uv = orc.observations(s)
    cf = T(s.cam_fixed, torch.uint8) if s.cam_fixed.any() else None
    ctx = ba.ba_create(s.n_cams, s.n_pts, T(s.obs_cam, torch.int32), T(s.obs_pt, torch.int32), T(uv, torch.float64),
                       cf, precision=ba.BA_MIXED)
    net = ba.ba_gnn_create(lp.load_weights(lp.DEFAULT_FSAI_WEIGHTS))
    r = {}
    try:
        r["pattern"] = digest(*ba.ba_get_pattern(ctx))
        cams, pts = T(s.cams_init, torch.float64), T(s.pts_init, torch.float64)
        ba.ba_linearize(ctx, cams, pts)
        ba.ba_form_rcs(ctx, 1e-3)
        r["rcs"] = digest(*ba.ba_get_rcs(ctx))
        dx = torch.empty((ba.ba_get_sizes(ctx)["n_rows"], 9), dtype=torch.float64, device=dev)
        ba.ba_set_preconditioner_net(ctx, net)
        for pre in (ba.BA_PRECOND_BLOCK_JACOBI, ba.BA_PRECOND_FSAI, ba.BA_PRECOND_LEARNED_FSAI):
            ba.ba_pcg_solve(ctx, dx, tol=1e-12, max_iter=5, precond=pre)
            r[f"pcg{pre}"] = digest(dx.cpu().numpy())
        ba.ba_lm_step(ctx, cams, pts, ba.new_lm_state(1e-4))
        r["lm"] = digest(cams.cpu().numpy(), pts.cpu().numpy())
    finally:
        ba.ba_set_preconditioner_net(ctx, None)
        ba.ba_gnn_destroy(net)
        ba.ba_destroy(ctx)
    return r


def shared(s):
    pu, pv = I.project(s.ext_true, s.intr_true, s.img_cam, s.pts_true, s.obs_img, s.obs_pt)
    uv = np.stack([pu.v, pv.v]) + s.noise
    ctx = ba.ba_create_shared(s.n_img, s.n_phys, s.n_pts, T(s.obs_img, torch.int32), T(s.obs_pt, torch.int32),
                              T(uv, torch.float64), T(s.img_cam, torch.int32), None)
    try:
        r = {"pattern": digest(*ba.ba_get_pattern(ctx))}
        params = T(np.concatenate([s.ext_init.ravel(), s.intr_init.ravel()]), torch.float64)
        ba.ba_linearize(ctx, params, T(s.pts_init, torch.float64))
        ba.ba_form_rcs(ctx, 1e-3)
        r["rcs"] = digest(*ba.ba_get_rcs(ctx))
    finally:
        ba.ba_destroy(ctx)
    return r


SCENES = {
    "aerial": lambda: nine(scenegen.aerial_grid_scene(seed=4, nx=10, ny=8, n_pts=20000, with_stats=False)),
    "long": lambda: nine(scenegen.long_track_scene()),
    "shared_long": lambda: shared(scenegen.shared_intrinsics_scene(seed=10, nx=10, ny=8, n_pts=400, n_phys=2,
                                                                   long_tracks=(65, 72, 80))),
}

if __name__ == "__main__":
    print(json.dumps({k: SCENES[k]() for k in sys.argv[1:]}), flush=True)
