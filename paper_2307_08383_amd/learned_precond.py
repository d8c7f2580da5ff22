"""Training and evaluation of the learned corrections of block-Jacobi.

RCS instances come from the method itself: LM runs of the library on seeded
aerial-grid scenes; after every LM iteration the context's RCS becomes a
training graph (network input built on the GPU).  Training runs the
library's own bf16 MFMA forward/backward kernels and Adam.  Two heads:
  block: per-camera correction of the block-Jacobi blocks (Hutchinson
         estimate of |B A - I|_F^2);
  fsai:  factorised correction M^-1 = G^T G on the FSAI pattern (exact
         Kaporin functional, minimised over the pattern by exact FSAI).
Evaluation compares PCG iteration counts and times on the same RCS, for
held-out scenes.

Usage (GPU):
  python -m paper_2307_08383_amd.learned_precond --head fsai --train-seeds 0-199 \
      --eval-seeds 200-219 --out paper_2307_08383_amd/learned_precond_fsai_weights.npy
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
DEFAULT_FSAI_WEIGHTS = os.path.join(HERE, "learned_precond_fsai_weights.npy")

# training scenes: the aerial-grid and partition generators at reduced
# extent (same camera spacing, overlap, point density and track law as the
# 2,000-camera and 60,000-camera scenes; the partition keeps its ring of
# fixed cameras)
TRAIN_GRID = dict(nx=20, ny=16, n_pts=64_000)
TRAIN_PARTITION = dict(nx=24, ny=20, n_pts=200_000)
# scene kinds for training and evaluation: small grids are dominated by
# border cameras, the larger ones by interior cameras (more neighbours)
KINDS = {
    "aerial": TRAIN_GRID,
    "aerial_full": dict(nx=50, ny=40, n_pts=400_000),
    "partition": ("partition", TRAIN_PARTITION),
    "partition_mid": ("partition", dict(nx=60, ny=50, n_pts=1_250_000)),
    "partition_big": ("partition", dict(nx=120, ny=100, n_pts=5_000_000)),
}


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
    # factorised head: hidden layer random, output layer zero (block-Jacobi)
    shapes += [(192, 128), (128,), (128, 96), (96,), (96,)]
    parts = []
    for i, sh in enumerate(shapes):
        if len(sh) == 2 and (i < n_trunk - 2 or i == n_trunk):
            scale = 0.5 if (sh[0] == 128 and i < n_trunk) else 1.0
            parts.append(rng.normal(0.0, scale / np.sqrt(sh[0]), size=sh).ravel())
        else:
            parts.append(np.zeros(int(np.prod(sh))))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == ba.ba_gnn_param_count()
    return w


def _scene(seed, grid):
    """grid: aerial-grid extent, or ("partition", extent)."""
    from . import scenegen
    if isinstance(grid, tuple):
        return scenegen.partition_scene(seed=seed, with_stats=False, **grid[1])
    return scenegen.aerial_grid_scene(seed=seed, with_stats=False, **grid)


def _context(scene, precision=0):
    import torch
    from . import ba
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    obs_cam, obs_pt = T(scene.obs_cam, torch.int32), T(scene.obs_pt, torch.int32)
    uv = ba.ba_project(T(scene.cams_true, torch.float64), T(scene.pts_true, torch.float64), obs_cam, obs_pt,
                       T(scene.noise, torch.float64))
    cf = T(scene.cam_fixed, torch.uint8) if scene.cam_fixed.any() else None
    ctx = ba.ba_create(scene.n_cams, scene.n_pts, obs_cam, obs_pt, uv, cf, precision=precision)
    return ctx, T(scene.cams_init, torch.float64), T(scene.pts_init, torch.float64)


def collect_graphs(seeds, grid=TRAIN_GRID, lm_iters=8, log=print, grids=None):
    """Network inputs of the RCS of every LM iteration of each scene (with
    grids, scene s uses grids[s % len(grids)])."""
    from . import ba
    graphs = []
    for s in seeds:
        scene = _scene(s, grids[s % len(grids)] if grids else grid)
        ctx, cams, pts = _context(scene)
        st = ba.new_lm_state(1e-4)
        for _ in range(lm_iters):
            ba.ba_lm_step(ctx, cams, pts, st)
            graphs.append(ba.ba_gnn_graph_from_ctx(ctx))
        ba.ba_destroy(ctx)
        log(f"scene {s}: {len(graphs)} graphs")
    return graphs


def train(net, graphs, epochs=6, batch=8, lr=1e-3, seed=0, log=print, head="block", cosine=False):
    """Adam steps over shuffled mini-batches; with cosine, the step size
    follows a half cosine from lr down to lr / 20 over the whole run."""
    from . import ba
    rng = np.random.default_rng(seed)
    hist = []
    step = 0
    n_steps = epochs * ((len(graphs) + batch - 1) // batch)
    for ep in range(epochs):
        order = rng.permutation(len(graphs))
        losses = []
        for b in range(0, len(order), batch):
            sel = [graphs[i] for i in order[b:b + batch]]
            lr_t = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * step / n_steps))) if cosine else lr
            if head == "fsai":
                losses.append(ba.ba_gnn_fsai_train_step(net, sel, lr=lr_t))
            else:
                losses.append(ba.ba_gnn_train_step(net, sel, n_probes=4, seed=int(rng.integers(1 << 62)), lr=lr_t))
            step += 1
        hist.append(float(np.mean(losses)))
        log(f"epoch {ep}: mean loss {hist[-1]:.6f} ({step} steps)")
    return hist


def evaluate(net, seeds, grid=TRAIN_GRID, lm_iters=8, tol=1e-6, max_iter=1000, log=print, head="block"):
    """PCG to rel tol on the RCS of each LM iteration (block-Jacobi LM
    trajectory) with block-Jacobi and the learned preconditioner; for the
    fsai head also exact FSAI, and both factorised ones with the gauge
    deflated."""
    import torch
    from . import ba
    if head == "fsai":
        variants = [("bj", ba.BA_PRECOND_BLOCK_JACOBI, False), ("fsai", ba.BA_PRECOND_FSAI, False),
                    ("learned", ba.BA_PRECOND_LEARNED_FSAI, False), ("fsai_defl", ba.BA_PRECOND_FSAI, True),
                    ("learned_defl", ba.BA_PRECOND_LEARNED_FSAI, True)]
    else:
        variants = [("bj", ba.BA_PRECOND_BLOCK_JACOBI, False), ("learned", ba.BA_PRECOND_LEARNED, False)]
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
            row = dict(seed=s, lm_iter=it)
            ref = None
            for name, pre, defl in variants:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = ba.ba_pcg_solve(ctx, dx, tol=tol, max_iter=max_iter, precond=pre, deflate=defl)
                torch.cuda.synchronize()
                row[name + "_iters"] = r["iters"]
                row[name + "_ms"] = r["ms"]
                # with the preconditioner's set-up on this RCS (network
                # inference, exact FSAI, deflation space)
                row[name + "_wall_ms"] = 1e3 * (time.perf_counter() - t0)
                row[name + "_capped"] = int(r["status"] == ba.BA_ERR_NOT_CONVERGED)
                if ref is None:
                    ref = dx.clone()
                else:
                    row[name + "_rel_diff"] = float(torch.linalg.norm(dx - ref) / torch.linalg.norm(ref))
            rows.append(row)
        ba.ba_set_preconditioner_net(ctx, None)
        ba.ba_destroy(ctx)
        last = rows[-lm_iters:]
        log(f"eval scene {s}: " + ", ".join(f"{n} {sum(r[n + '_iters'] for r in last)} it"
                                            for n, _, _ in variants))
    out = dict(rows=rows)
    for name, _, _ in variants:
        out[name + "_iters"] = sum(r[name + "_iters"] for r in rows)
        out[name + "_ms"] = sum(r[name + "_ms"] for r in rows)
        out[name + "_wall_ms"] = sum(r[name + "_wall_ms"] for r in rows)
        out[name + "_capped"] = sum(r[name + "_capped"] for r in rows)
    out["iter_ratio"] = out["learned_iters"] / max(out["bj_iters"], 1)
    return out


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
    ap.add_argument("--head", default="block", choices=["block", "fsai"])
    ap.add_argument("--train-seeds", default="0-199")
    ap.add_argument("--eval-seeds", default="200-219")
    ap.add_argument("--lm-iters", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--cosine", action="store_true", help="half-cosine step-size decay to lr / 20")
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None)
    ap.add_argument("--eval-full-seeds", default="",
                    help="held-out seeds evaluated on the full 50 x 40 aerial grid as well")
    ap.add_argument("--kinds", default="aerial", help="training scene kinds, comma separated: " + ", ".join(KINDS))
    ap.add_argument("--eval-kinds", default="", help="scene kinds evaluated on held-out seeds (default: --kinds)")
    ap.add_argument("--eval-only", action="store_true",
                    help="no training: evaluate the weights of --weights (default: the head's shipped weights)")
    ap.add_argument("--weights", default=None)
    args = ap.parse_args()
    from . import ba
    out = args.out or (DEFAULT_FSAI_WEIGHTS if args.head == "fsai" else DEFAULT_WEIGHTS)
    log = lambda m: print(m, flush=True)
    t0 = time.time()
    if args.eval_only:
        import torch
        torch.zeros(1, device="cuda")   # torch's device context before the library's first call
        wpath = args.weights or (DEFAULT_FSAI_WEIGHTS if args.head == "fsai" else DEFAULT_WEIGHTS)
        net = ba.ba_gnn_create(load_weights(wpath))
        rep = dict(head=args.head, weights=os.path.basename(wpath), eval_seeds=args.eval_seeds,
                   lm_iters=args.lm_iters)
        for k in (args.eval_kinds or "aerial_full").split(","):
            ev = evaluate(net, _range(args.eval_seeds), grid=KINDS[k], lm_iters=args.lm_iters, log=log,
                          head=args.head)
            rep["eval_" + k] = dict((kk, v) for kk, v in ev.items() if kk != "rows")
            rep["eval_" + k + "_rows"] = ev["rows"]
            log(json.dumps(rep["eval_" + k]))
        ba.ba_gnn_destroy(net)
        if args.report:
            with open(args.report, "w") as f:
                json.dump(rep, f, indent=1)
        log(f"evaluated in {time.time() - t0:.1f} s")
        return
    kinds = args.kinds.split(",")
    grids = [KINDS[k] for k in kinds]
    graphs = collect_graphs(_range(args.train_seeds), lm_iters=args.lm_iters, log=log, grids=grids)
    log(f"collected {len(graphs)} graphs in {time.time() - t0:.1f} s")
    net = ba.ba_gnn_create(init_params(0))
    t1 = time.time()
    hist = train(net, graphs, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log, head=args.head,
                 cosine=args.cosine)
    log(f"trained in {time.time() - t1:.1f} s")
    for g in graphs:
        ba.ba_gnn_graph_destroy(g)
    w = ba.ba_gnn_get_params(net)
    np.save(out, w, allow_pickle=False)
    rep = dict(head=args.head, kinds=kinds, grids={k: KINDS[k] for k in kinds}, train_seeds=args.train_seeds,
               eval_seeds=args.eval_seeds, lm_iters=args.lm_iters, epochs=args.epochs, batch=args.batch,
               lr=args.lr, cosine=args.cosine, loss_history=hist)
    eval_kinds = args.eval_kinds.split(",") if args.eval_kinds else kinds
    for k in eval_kinds:
        ev = evaluate(net, _range(args.eval_seeds), grid=KINDS[k], lm_iters=args.lm_iters, log=log, head=args.head)
        rep["eval_" + k] = dict((kk, v) for kk, v in ev.items() if kk != "rows")
        rep["eval_" + k + "_rows"] = ev["rows"]
    rep["eval"] = rep["eval_" + eval_kinds[0]]
    if args.eval_full_seeds:
        full = dict(nx=50, ny=40, n_pts=400_000)
        evf = evaluate(net, _range(args.eval_full_seeds), grid=full, lm_iters=args.lm_iters, log=log, head=args.head)
        rep["eval_full"] = dict((k, v) for k, v in evf.items() if k != "rows")
        rep["eval_full_rows"] = evf["rows"]
    ba.ba_gnn_destroy(net)
    log(json.dumps(rep["eval"]))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
