"""Training and evaluation of the learned block-Jacobi correction.

RCS instances come from the method itself: LM runs of the library on seeded
aerial-grid scenes; after every LM iteration the context's RCS becomes a
training graph (network input built on the GPU).  Training runs the
library's own bf16 MFMA forward/backward kernels and Adam.  Evaluation
compares PCG iteration counts and times with block-Jacobi and with the
learned preconditioner on the same RCS, for held-out scenes.

Usage (GPU):
  python -m paper_2307_08383_amd.learned_precond --train-seeds 0-199 \
      --eval-seeds 200-219 --out paper_2307_08383_amd/learned_precond_weights.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

DEFAULT_WEIGHTS = os.path.join(HERE, "learned_precond_weights.npy")

# training scene: the aerial-grid generator at reduced extent (same camera
# spacing, overlap, point density and track law as the 2,000-camera scene)
TRAIN_GRID = dict(nx=20, ny=16, n_pts=64_000)


def init_params(seed=0):
    """Initial parameters: random encoder/message/update weights with std
    1/sqrt(fan_in) (update layers halved), zero biases, zero decoder (the
    network starts as exact block-Jacobi)."""
    from . import ba
    rng = np.random.default_rng(seed)
    shapes = [(64, 64), (64,), (96, 64), (64,)]
    for _ in range(3):
        shapes += [(192, 64), (64,), (128, 64), (64,)]
    shapes += [(64, 48), (48,)]
    n_trunk = len(shapes)
    shapes += [(192, 96), (96,), (96,)]       # factorised head (zero: block-Jacobi)
    parts = []
    for i, sh in enumerate(shapes):
        if len(sh) == 2 and i < n_trunk - 2:
            scale = 0.5 if sh[0] == 128 else 1.0
            parts.append(rng.normal(0.0, scale / np.sqrt(sh[0]), size=sh).ravel())
        else:
            parts.append(np.zeros(int(np.prod(sh))))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == ba.ba_gnn_param_count()
    return w


def _scene(seed, grid):
    from . import scenegen
    return scenegen.aerial_grid_scene(seed=seed, with_stats=False, **grid)


def _context(scene, precision=0):
    import torch
    from . import ba
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    obs_cam, obs_pt = T(scene.obs_cam, torch.int32), T(scene.obs_pt, torch.int32)
    uv = ba.ba_project(T(scene.cams_true, torch.float64), T(scene.pts_true, torch.float64), obs_cam, obs_pt,
                       T(scene.noise, torch.float64))
    ctx = ba.ba_create(scene.n_cams, scene.n_pts, obs_cam, obs_pt, uv, precision=precision)
    return ctx, T(scene.cams_init, torch.float64), T(scene.pts_init, torch.float64)


def collect_graphs(seeds, grid=TRAIN_GRID, lm_iters=8, log=print):
    """Network inputs of the RCS of every LM iteration of each scene."""
    from . import ba
    graphs = []
    for s in seeds:
        scene = _scene(s, grid)
        ctx, cams, pts = _context(scene)
        st = ba.new_lm_state(1e-4)
        for _ in range(lm_iters):
            ba.ba_lm_step(ctx, cams, pts, st)
            graphs.append(ba.ba_gnn_graph_from_ctx(ctx))
        ba.ba_destroy(ctx)
        log(f"scene {s}: {len(graphs)} graphs")
    return graphs


def train(net, graphs, epochs=6, batch=8, lr=1e-3, seed=0, log=print):
    from . import ba
    rng = np.random.default_rng(seed)
    hist = []
    step = 0
    for ep in range(epochs):
        order = rng.permutation(len(graphs))
        losses = []
        for b in range(0, len(order), batch):
            sel = [graphs[i] for i in order[b:b + batch]]
            losses.append(ba.ba_gnn_train_step(net, sel, n_probes=4, seed=int(rng.integers(1 << 62)), lr=lr))
            step += 1
        hist.append(float(np.mean(losses)))
        log(f"epoch {ep}: mean loss {hist[-1]:.6f} ({step} steps)")
    return hist


def evaluate(net, seeds, grid=TRAIN_GRID, lm_iters=8, tol=1e-6, max_iter=1000, log=print):
    """PCG to rel tol on the RCS of each LM iteration (block-Jacobi LM
    trajectory), with block-Jacobi and with the learned preconditioner."""
    import torch
    from . import ba
    rows = []
    for s in seeds:
        scene = _scene(s, grid)
        ctx, cams, pts = _context(scene)
        ba.ba_set_preconditioner_net(ctx, net)
        n_rows = ba.ba_get_sizes(ctx)["n_rows"]
        dx = torch.empty((n_rows, 9), dtype=torch.float64, device="cuda")
        st = ba.new_lm_state(1e-4)
        for it in range(lm_iters):
            ba.ba_lm_step(ctx, cams, pts, st)
            a = ba.ba_pcg_solve(ctx, dx, tol=tol, max_iter=max_iter)
            xa = dx.clone()
            b = ba.ba_pcg_solve(ctx, dx, tol=tol, max_iter=max_iter, precond=ba.BA_PRECOND_LEARNED)
            err = float(torch.linalg.norm(dx - xa) / torch.linalg.norm(xa))
            rows.append(dict(seed=s, lm_iter=it, bj_iters=a["iters"], learned_iters=b["iters"],
                             bj_ms=a["ms"], learned_ms=b["ms"], rel_diff=err))
        ba.ba_set_preconditioner_net(ctx, None)
        ba.ba_destroy(ctx)
        last = rows[-lm_iters:]
        log(f"eval scene {s}: BJ {sum(r['bj_iters'] for r in last)} it, "
            f"learned {sum(r['learned_iters'] for r in last)} it")
    bj = sum(r["bj_iters"] for r in rows)
    le = sum(r["learned_iters"] for r in rows)
    return dict(rows=rows, bj_iters=bj, learned_iters=le, iter_ratio=le / max(bj, 1),
                bj_ms=sum(r["bj_ms"] for r in rows), learned_ms=sum(r["learned_ms"] for r in rows))


def load_weights(path=DEFAULT_WEIGHTS):
    """Parameters from a .npy file; a file without the factorised head
    (older, shorter parameter vector) gets a zero head."""
    from . import ba
    w = np.load(path, allow_pickle=False).astype(np.float32)
    n = ba.ba_gnn_param_count()
    if w.size < n:
        w = np.concatenate([w, np.zeros(n - w.size, np.float32)])
    return w


def _range(spec):
    a, b = spec.split("-") if "-" in spec else (spec, spec)
    return list(range(int(a), int(b) + 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-seeds", default="0-199")
    ap.add_argument("--eval-seeds", default="200-219")
    ap.add_argument("--lm-iters", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    from . import ba
    log = lambda m: print(m, flush=True)
    t0 = time.time()
    graphs = collect_graphs(_range(args.train_seeds), lm_iters=args.lm_iters, log=log)
    log(f"collected {len(graphs)} graphs in {time.time() - t0:.1f} s")
    net = ba.ba_gnn_create(init_params(0))
    t1 = time.time()
    hist = train(net, graphs, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    log(f"trained in {time.time() - t1:.1f} s")
    for g in graphs:
        ba.ba_gnn_graph_destroy(g)
    w = ba.ba_gnn_get_params(net)
    np.save(args.out, w, allow_pickle=False)
    ev = evaluate(net, _range(args.eval_seeds), lm_iters=args.lm_iters, log=log)
    ba.ba_gnn_destroy(net)
    rep = dict(train_seeds=args.train_seeds, eval_seeds=args.eval_seeds, lm_iters=args.lm_iters,
               epochs=args.epochs, batch=args.batch, lr=args.lr, grid=TRAIN_GRID, loss_history=hist,
               eval=dict((k, v) for k, v in ev.items() if k != "rows"), eval_rows=ev["rows"])
    log(json.dumps(rep["eval"]))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
