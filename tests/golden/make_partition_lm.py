"""Writes partition60000_lm_oracle.json: the oracle's fixed-budget LM run on
the 60,000-camera partition scene (seed 2: 25M points, ~100M observations,
a ring of fixed cameras), the one-GPU share that the learned-vs-block-Jacobi
comparison is defined on.

Calls only the scene generator (random draws) and the oracle: observations
= the oracle's projection of the true parameters plus the scene's noise;
10 LM iterations from the perturbed start, lambda0 = 1e-4, block-Jacobi PCG
to rel 1e-6 with at most 1000 iterations (Sec. 3.1 Eq. (1), Eq. (4)-(7), (5);
the damping schedule is the reading the oracle takes).  The oracle holds
about 40 GB of host memory on this scene and takes 20-30 minutes on 8 cores.

Usage: python tests/golden/make_partition_lm.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as orc  # noqa: E402
from paper_2307_08383_amd import scenegen  # noqa: E402

OUT = os.path.join(HERE, "partition60000_lm_oracle.json")


def run(scene, out_path, about, pcg_tol=None, pcg_max_iter=1000):
    """The oracle's fixed-budget LM run on `scene` (block-Jacobi PCG to
    pcg_tol, by default the scene's tolerance, at most pcg_max_iter
    iterations; lambda0 1e-4), stored with the scene's digest and the digest
    of the observations it was run on."""
    t0 = time.time()
    s = scene
    uv = orc.observations(s)
    uv_sha = hashlib.sha256(np.ascontiguousarray(uv).tobytes()).hexdigest()
    print(f"scene {s.name}: {s.n_obs} observations ({time.time() - t0:.0f} s)", flush=True)
    P = orc.Problem.from_scene(s, uv)
    cams = np.array(s.cams_init, dtype=np.float64, order="C")
    pts = np.array(s.pts_init, dtype=np.float64, order="C")
    st = orc.LMState(lam=1e-4, nu=2.0, iter=0, pad=0)
    hist = []
    for it in range(s.lm_iterations):
        t1 = time.time()
        lam_before, nu_before = st.lam, st.nu
        info = P.lm_step(cams, pts, st, s.pcg_tol if pcg_tol is None else pcg_tol, pcg_max_iter)
        info.update(lambda_before=lam_before, nu_before=nu_before, lambda_after=st.lam, nu_after=st.nu,
                    seconds=time.time() - t1)
        hist.append(info)
        print(f"iteration {it}: F {info['cost']:.10e} F' {info['cost_new']:.10e} accepted {info['accepted']} "
              f"pcg {info['pcg_iters']} relres {info['pcg_relres']:.2e} ({info['seconds']:.0f} s)", flush=True)
        if info["stop"]:
            break
    F_final = P.cost(cams, pts)
    out = dict(about=about, scene=s.name, scene_digest=s.digest(), uv_sha256=uv_sha, n_obs=s.n_obs,
               pcg_tol=s.pcg_tol if pcg_tol is None else pcg_tol, pcg_max_iter=pcg_max_iter,
               oracle_threads=orc.default_threads(), iterations=hist, final_cost=F_final,
               wall_seconds=time.time() - t0)
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"final cost {F_final:.12e}; wrote {out_path}", flush=True)


def main():
    run(scenegen.partition_scene(seed=2, with_stats=False), OUT,
        "Oracle (FP64, CPU) LM run on the 60,000-camera partition scene (seed 2): 10 iterations "
        "from the perturbed start, lambda0 1e-4, block-Jacobi PCG to rel 1e-6, cap 1000. "
        "Written by tests/golden/make_partition_lm.py from the oracle only.")


if __name__ == "__main__":
    main()
