"""Benchmark of the bundle-adjustment hot path on one MI355X.

A step is one LM iteration (linearize, RCS formation, block-Jacobi PCG to
rel 1e-6, back-substitution, candidate cost and gain ratio).  The default
workload is the one-GPU share of the 1M-camera problem: a 60,000-camera
partition with a ring of fixed cameras of neighbouring partitions, 25M
points, track length truncated-geometric on [2, 12] with mean 4 (~100M
observations), pixel noise N(0, 0.5^2), FP64.  Inputs are synthetic and
resident in HBM before timing starts.

Printed JSON line: value = RCS formation throughput (observations per
second through the fused linearize + point stage, the camera-pair stage and
the diagonal stage; device time of the timed steps that relinearize);
ms_per_step = LM-iteration wall time; the roofline entry covers the
formation kernel that takes the most time, with the others beside it;
cpu_baseline is the C oracle on the host cores for a bounded sample (a
smaller partition from the same generator): its formation rate and its
LM-iteration time.  lm_comparison: LM runs of the learned + mixed variants
against plain FP64 block-Jacobi on the same scene for the scene's budget
(10 LM iterations), with per-solve residuals and total time to the final
cost.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RCS formation obs/s + LM-iteration time, learned vs block-Jacobi PCG"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="partition", choices=["aerial", "strips", "partition"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default="partition-2400",
                    choices=["partition-2400", "partition-600", "aerial"],
                    help="scene the oracle is timed on: a 50 x 48 (or 25 x 24) partition from the same "
                         "generator as the default workload, or the 2,000-camera aerial scene")
    ap.add_argument("--cpu-lm-iters", type=int, default=2, help="oracle LM iterations timed on the sample")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the learned + mixed vs FP64 block-Jacobi LM comparison")
    ap.add_argument("--lm-iters", type=int, default=None,
                    help="LM iterations of each compared run (default: the workload's budget)")
    ap.add_argument("--compare", default="default",
                    help="comma-separated subset of the compared runs, 'default' or 'all'")
    ap.add_argument("--precond", default="block_jacobi",
                    choices=["block_jacobi", "fsai", "learned", "learned_fsai"],
                    help="preconditioner of the timed LM steps")
    ap.add_argument("--deflate", action="store_true", help="gauge-deflated PCG in the timed LM steps")
    ap.add_argument("--aerial-compare", action="store_true",
                    help="also run the LM comparison on the 2,000-camera aerial scene")
    ap.add_argument("--solver-fp32", action="store_true",
                    help="PCG products on an FP32 copy of S in the timed LM steps")
    ap.add_argument("--product", default="auto", choices=["auto", "full", "upper"],
                    help="layout of the PCG product S z in the timed LM steps and the comparisons")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first, so that hardware "
                         "byte counters can be scaled against a kernel of known traffic")
    return ap.parse_args()


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_scene(kind):
    from paper_2307_08383_amd import scenegen
    if kind == "aerial":
        return scenegen.aerial_grid_scene(seed=0, with_stats=False)
    if kind == "strips":
        return scenegen.strips_scene(seed=1, with_stats=False)
    if kind == "partition-2400":
        return scenegen.partition_scene(seed=2, nx=50, ny=48, n_pts=1_000_000)
    if kind == "partition-600":
        return scenegen.partition_scene(seed=2, nx=25, ny=24, n_pts=250_000)
    return scenegen.partition_scene(seed=2, with_stats=False)


def stage_bytes(scene, sizes, precision):
    """Algorithmic HBM bytes of one launch of each formation kernel (the
    minimum each must move; per-unit counts of the kernels' design):
      linpoint (linearize + point stage) per observation: indices, pixels and
        camera-list slot 28, records J_c + K 24 (x sizeof T), e 16,
        e + K lhat 16; per point: its parameters 24 and point terms 72 (J_p
        is not stored: it is K L^T);
      pair per observation couple: two indices 8 and two records 2 x 24
        (x sizeof T); per off-diagonal block: 81 FP64 values and its bounds 8;
      diag per observation of a free camera: its list entry 4, record 24
        (x sizeof T), e + K lhat 16; per RCS row: the diagonal block, the
        block-Jacobi inverse and L^-1 (3 x 81 FP64), rhs 72 and bounds 12."""
    es = 4 if precision == "mixed" else 8
    n, npt = scene.n_obs, scene.n_pts
    free_obs = int((~scene.cam_fixed.astype(bool))[scene.obs_cam].sum())
    n_offseg = sizes["n_blk"] - sizes["n_rows"]
    return {"linpoint": n * (28 + 24 * es + 16 + 16) + npt * (24 + 72),
            "pair": sizes["n_pairs"] * (8 + 2 * 24 * es) + n_offseg * (81 * 8 + 8),
            "diag": free_obs * (4 + 24 * es + 16) + sizes["n_rows"] * (3 * 81 * 8 + 72 + 12)}


KERNEL_OF_STAGE = {"linpoint": {"fp64": "k_linpoint_d", "mixed": "k_linpoint_f"},
                   "pair": {"fp64": "k_offdiag<double>", "mixed": "k_offdiag<float>"},
                   "diag": {"fp64": "k_diag<double>", "mixed": "k_diag<float>"}}


def formation_source_hash():
    h = hashlib.sha256()
    for f in ("kernels_rcs.hip", "ba_common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2307_08383_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_from_profile(key):
    """HBM traffic per launch from committed rocprofv3 counter summaries, if
    they were taken on the current formation kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        ent = json.load(open(path)).get(key)
        if ent and ent.get("source_sha256") == formation_source_hash():
            return ent.get("bytes_per_launch")
    except Exception:
        return None
    return None


def _relin_flags(st):
    return not (st.flags & 1)


def lm_run(scene, obs, precision, precond, iters, learned_weights=None, deflate=False, solver_fp32=False,
           product=0):
    """LM run from the scene's start; returns per-iteration means, per-solve
    residuals, the total time to the final cost (with the first-use set-up)
    and the final cost (FP64 cost of the last iterate)."""
    import torch
    from paper_2307_08383_amd import ba
    obs_cam, obs_pt, uv, cf = obs
    torch.cuda.synchronize()
    t_c = time.perf_counter()
    ctx = ba.ba_create(scene.n_cams, scene.n_pts, obs_cam, obs_pt, uv, cf, precision=precision)
    torch.cuda.synchronize()
    create_ms = 1e3 * (time.perf_counter() - t_c)
    dev = uv.device
    cams = torch.as_tensor(scene.cams_init, dtype=torch.float64, device=dev).contiguous()
    pts = torch.as_tensor(scene.pts_init, dtype=torch.float64, device=dev).contiguous()
    # one-time structures built on first use (the network's graph, index sets
    # of the FSAI pattern, the FP32 copy), like the co-visibility pattern at
    # creation: built here, outside the timed run, from a formed RCS at the
    # start point (parameters unchanged), and reported separately
    setup_ms = 0.0
    net = None
    if precond != ba.BA_PRECOND_BLOCK_JACOBI or deflate or solver_fp32:
        torch.cuda.synchronize()
        t_s = time.perf_counter()
        if precond in (ba.BA_PRECOND_LEARNED, ba.BA_PRECOND_LEARNED_FSAI):
            net = ba.ba_gnn_create(learned_weights)
            ba.ba_set_preconditioner_net(ctx, net)
        ba.ba_linearize(ctx, cams, pts)
        ba.ba_form_rcs(ctx, 1e-4)
        dx = torch.empty((ba.ba_get_sizes(ctx)["n_rows"], 9), dtype=torch.float64, device=dev)
        ba.ba_pcg_solve(ctx, dx, tol=scene.pcg_tol, max_iter=1, precond=precond, deflate=deflate,
                        solver_fp32=solver_fp32, product=product)
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t_s)
    st = ba.new_lm_state(1e-4)
    infos, relin = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        relin.append(_relin_flags(st))
        infos.append(ba.ba_lm_step(ctx, cams, pts, st, pcg_tol=scene.pcg_tol, precond=precond, deflate=deflate,
                                   solver_fp32=solver_fp32, product=product))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # FP64 cost of the final parameters (the mixed path evaluates cost in FP64 too)
    final = ba.ba_linearize(ctx, cams, pts)
    if net is not None:
        ba.ba_set_preconditioner_net(ctx, None)
        ba.ba_gnn_destroy(net)
    ba.ba_destroy(ctx)
    form = [i["ms_linearize"] + i["ms_form_rcs"] for i, r in zip(infos, relin) if r]
    return dict(ms_per_iter=1e3 * wall / iters, total_ms_to_final_cost=1e3 * wall + setup_ms,
                final_cost=final, first_use_setup_ms=setup_ms, create_ms=create_ms,
                accepted=int(sum(i["accepted"] for i in infos)),
                pcg_iters=[int(i["pcg_iters"]) for i in infos],
                pcg_relres=[float(i["pcg_relres"]) for i in infos],
                pcg_capped=int(sum(i["pcg_status"] == ba.BA_ERR_NOT_CONVERGED for i in infos)),
                precond_fallbacks=int(sum(i["precond_fallback"] for i in infos)),
                pcg_iters_mean=float(np.mean([i["pcg_iters"] for i in infos])),
                precond_ms_mean=float(np.mean([i["ms_precond"] for i in infos])),
                formation_ms_mean=float(np.mean(form)) if form else None,
                formation_obs_per_s=scene.n_obs / (1e-3 * float(np.mean(form))) if form else None,
                pcg_ms_mean=float(np.mean([i["ms_pcg"] for i in infos])))


def device_observations(scene, dev):
    """Observations on the device: indices, pixels = projection of the true
    parameters + the scene's noise (by the library's own projection), fixed
    camera flags (or None)."""
    import torch
    from paper_2307_08383_amd import ba
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    obs_cam = T(scene.obs_cam, torch.int32)
    obs_pt = T(scene.obs_pt, torch.int32)
    uv = ba.ba_project(T(scene.cams_true, torch.float64), T(scene.pts_true, torch.float64),
                       obs_cam, obs_pt, T(scene.noise, torch.float64))
    cf = T(scene.cam_fixed, torch.uint8) if scene.cam_fixed.any() else None
    return obs_cam, obs_pt, uv, cf


# variants of the LM comparison: name, precision, preconditioner, deflation
# (the "_s32_" ones run the solver's products on an FP32 copy of S)
PRODUCTS = {"auto": 0, "full": 1, "upper": 2}   # BA_PRODUCT_*

COMPARE_VARIANTS = [
    ("fp64_block_jacobi", "fp64", "block_jacobi", False),
    ("mixed_block_jacobi", "mixed", "block_jacobi", False),
    ("mixed_block_jacobi_deflated", "mixed", "block_jacobi", True),
    ("mixed_fsai", "mixed", "fsai", False),
    ("mixed_fsai_deflated", "mixed", "fsai", True),
    ("mixed_learned_block_deflated", "mixed", "learned", True),
    ("mixed_learned_fsai", "mixed", "learned_fsai", False),
    ("mixed_learned_fsai_deflated", "mixed", "learned_fsai", True),
    ("mixed_s32_block_jacobi_deflated", "mixed", "block_jacobi", True),
    ("mixed_s32_fsai_deflated", "mixed", "fsai", True),
    ("mixed_s32_learned_fsai_deflated", "mixed", "learned_fsai", True)]
# the default subset: plain FP64 block-Jacobi (the paper's solver), the
# mixed path alone, the learned factor with and without the non-learned
# extensions, and the same extensions without the network
DEFAULT_VARIANTS = ["fp64_block_jacobi", "mixed_block_jacobi", "mixed_learned_fsai",
                    "mixed_block_jacobi_deflated", "mixed_fsai_deflated", "mixed_learned_fsai_deflated",
                    "mixed_s32_block_jacobi_deflated", "mixed_s32_learned_fsai_deflated"]


def lm_comparison(scene, obs, names, lm_iters, product=0):
    """Each named variant from the scene's start for lm_iters LM iterations;
    ms per iteration, total time to the final cost, final FP64 cost and the
    ratios to FP64 block-Jacobi."""
    from paper_2307_08383_amd import ba
    from paper_2307_08383_amd import learned_precond as lp

    def weights(path):
        return (lp.load_weights(path), os.path.basename(path)) if os.path.exists(path) else \
            (lp.init_params(0), "untrained (zero head: block-Jacobi)")
    wb, wb_name = weights(lp.DEFAULT_WEIGHTS)
    wf, wf_name = weights(lp.DEFAULT_FSAI_WEIGHTS)
    pre_of = {"block_jacobi": ba.BA_PRECOND_BLOCK_JACOBI, "fsai": ba.BA_PRECOND_FSAI,
              "learned": ba.BA_PRECOND_LEARNED, "learned_fsai": ba.BA_PRECOND_LEARNED_FSAI}
    w_of = {"learned": wb, "learned_fsai": wf}
    runs = {}
    for name, precision, precond, defl in COMPARE_VARIANTS:
        if name not in names and name != "fp64_block_jacobi":
            continue
        prec = ba.BA_MIXED if precision == "mixed" else ba.BA_FP64
        runs[name] = lm_run(scene, obs, prec, pre_of[precond], lm_iters, w_of.get(precond), deflate=defl,
                            solver_fp32="_s32_" in name, product=product)
        progress(f"LM comparison {scene.name} {name}: {runs[name]['ms_per_iter']:.2f} ms per iteration, "
                 f"{runs[name]['pcg_capped']} capped solves")
    base = runs["fp64_block_jacobi"]
    return {
        "scene": scene.name, "n_obs": scene.n_obs, "iterations": lm_iters,
        **runs,
        "learned_weights": {"block": wb_name, "fsai": wf_name},
        "speedup_vs_fp64_block_jacobi": {k: base["ms_per_iter"] / v["ms_per_iter"] for k, v in runs.items()},
        "speedup_to_final_cost_with_setup_vs_fp64_block_jacobi": {
            k: base["total_ms_to_final_cost"] / v["total_ms_to_final_cost"] for k, v in runs.items()},
        "final_cost_rel_diff_vs_fp64_block_jacobi": {
            k: abs(v["final_cost"] - base["final_cost"]) / base["final_cost"] for k, v in runs.items()},
    }


def roofline_entry(kernel, alg_bytes, ms, traffic):
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes,
            "launch_ms": ms}


def storage_comparison(ctx, n_rows, dev, reps=20):
    """BSMC against scalar CSR on the RCS just formed (Sec. 4.1 Eq. (8)-(10)):
    bytes each layout holds and the device time of one product S x (median
    of `reps` event-timed calls on the context stream) for the two block
    layouts of the PCG product and the CSR copy."""
    import torch
    from paper_2307_08383_amd import ba
    sz = ba.ba_get_store_sizes(ctx)
    x = torch.randn((n_rows, 9), dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    out = {"bytes": {"bsmc_upper": sz["bsmc_bytes"], "full_copy": sz["full_bytes"], "csr": sz["csr_bytes"]},
           "csr_nnz": sz["csr_nnz"], "csr_over_bsmc_bytes": sz["csr_bytes"] / sz["bsmc_bytes"]}
    n_blk = (sz["csr_nnz"] // 81 + n_rows) // 2
    alpha = (2 * n_blk - n_rows) / n_rows ** 2
    n, c = n_rows, 9
    out["eq10_ratio"] = (6 * alpha * n * c * c + 2 * c) / (2 * alpha * n * c * c + 2 * c * c + 3 * alpha * n + 5)
    # bytes one product must read or write: UPPER reads each upper block and
    # its column index once and writes + reads a 9-vector per block; FULL
    # reads both triangles; CSR reads its values, columns and row pointer
    vec = 2 * 9 * n_rows * 8
    moved = {"upper": sz["bsmc_bytes"] + n_blk * 2 * 72 + vec, "full": sz["full_bytes"] + vec,
             "csr": sz["csr_bytes"] + vec}
    ms = {}
    for name, prod in (("upper", ba.BA_PRODUCT_UPPER), ("full", ba.BA_PRODUCT_FULL), ("csr", ba.BA_PRODUCT_CSR)):
        ba.ba_rcs_product(ctx, x, y, product=prod)   # builds the layout's copy on first use
        t = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            ba.ba_rcs_product(ctx, x, y, product=prod)
            b.record()
            b.synchronize()
            t.append(a.elapsed_time(b))
        ms[name] = float(np.median(t))
    out["product_ms"] = ms
    out["product_gbs"] = {k: moved[k] / (ms[k] * 1e-3) / 1e9 for k in ms}
    out["csr_over_bsmc_upper_time"] = ms["csr"] / ms["upper"]
    return out


def copy_peak_gbs(dev, mib=2048, reps=5):
    """Measured streaming bandwidth: the best of `reps` device copies of
    `mib` MiB (bytes read + written per copy), timed with events."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * mib * (1 << 20) / (best * 1e-3) / 1e9


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(kind, lm_iters, n_obs_workload):
    """The oracle (plain FP64 C, OpenMP) on a bounded sample: a smaller
    scene of the workload's generator.  Formation (linearize + RCS) on all
    host threads (two runs) and on one thread, then LM iterations from the
    start (block-Jacobi PCG to rel 1e-6, cap 1000) on all threads."""
    from oracle import oracle as orc
    s = build_scene(kind)
    nt = orc.default_threads()
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv, n_threads=nt)
    t0 = time.perf_counter()
    for _ in range(2):
        P.linearize(s.cams_init, s.pts_init)
        P.form_rcs(1e-4)
    dt = (time.perf_counter() - t0) / 2
    P1 = orc.Problem.from_scene(s, uv, n_threads=1)
    t1 = time.perf_counter()
    P1.linearize(s.cams_init, s.pts_init)
    P1.form_rcs(1e-4)
    dt1 = time.perf_counter() - t1
    del P1
    cams = np.array(s.cams_init, order="C")
    pts = np.array(s.pts_init, order="C")
    st = orc.LMState(lam=1e-4, nu=2.0, iter=0, pad=0)
    t2 = time.perf_counter()
    its = [P.lm_step(cams, pts, st, s.pcg_tol, 1000) for _ in range(lm_iters)]
    dt2 = (time.perf_counter() - t2) / lm_iters
    return {"value": s.n_obs / dt, "unit": "obs/s", "cores": nt, "kind": "oracle",
            "sample": f"{s.name} (same generator as the workload, {s.n_cams} cameras incl. the fixed ring, "
                      f"{s.n_obs} observations): formation (linearize + RCS) on {nt} threads, mean of 2 runs "
                      f"{dt:.2f} s; {lm_iters} LM iterations {dt2:.2f} s each",
            "single_thread_value": s.n_obs / dt1,
            "lm_iteration_s": dt2, "lm_pcg_iters": [int(i["pcg_iters"]) for i in its],
            "lm_iteration_s_per_obs": dt2 / s.n_obs,
            "lm_iteration_s_scaled_to_workload": dt2 / s.n_obs * n_obs_workload,
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library covers the one-GPU share of the "
              "problem and uses no collectives; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2307_08383_amd import ba

    dev = torch.device("cuda:0")
    scene = build_scene(args.workload)
    progress(f"scene {scene.name}: {scene.n_obs} observations")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    obs_cam, obs_pt, uv, cf = device_observations(scene, dev)
    prec = ba.BA_MIXED if args.precision == "mixed" else ba.BA_FP64
    torch.cuda.synchronize()
    t_c = time.perf_counter()
    ctx = ba.ba_create(scene.n_cams, scene.n_pts, obs_cam, obs_pt, uv, cf, precision=prec)
    torch.cuda.synchronize()
    create_ms = 1e3 * (time.perf_counter() - t_c)
    sizes = ba.ba_get_sizes(ctx)
    progress(f"context created: {sizes['n_blk']} blocks, {sizes['n_pairs']} observation couples")
    cams = T(scene.cams_init, torch.float64)
    pts = T(scene.pts_init, torch.float64)
    st = ba.new_lm_state(1e-4)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src_buf = torch.ones(n, dtype=torch.float64, device=dev)
        dst_buf = torch.empty_like(src_buf)
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        del src_buf, dst_buf
    pre = {"block_jacobi": ba.BA_PRECOND_BLOCK_JACOBI, "fsai": ba.BA_PRECOND_FSAI,
           "learned": ba.BA_PRECOND_LEARNED, "learned_fsai": ba.BA_PRECOND_LEARNED_FSAI}[args.precond]
    net = None
    if pre in (ba.BA_PRECOND_LEARNED, ba.BA_PRECOND_LEARNED_FSAI):
        from paper_2307_08383_amd import learned_precond
        net = ba.ba_gnn_create(learned_precond.load_weights(
            learned_precond.DEFAULT_FSAI_WEIGHTS if pre == ba.BA_PRECOND_LEARNED_FSAI else learned_precond.DEFAULT_WEIGHTS))
        ba.ba_set_preconditioner_net(ctx, net)
    step_kw = dict(pcg_tol=scene.pcg_tol, precond=pre, deflate=args.deflate, solver_fp32=args.solver_fp32,
                   product=PRODUCTS[args.product])
    for _ in range(args.warmup):
        ba.ba_lm_step(ctx, cams, pts, st, **step_kw)
    torch.cuda.synchronize()
    progress("warm-up done")
    infos, stages, relin = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        relin.append(_relin_flags(st))
        infos.append(ba.ba_lm_step(ctx, cams, pts, st, **step_kw))
        stages.append(ba.ba_get_stage_ms(ctx))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    # formation of a relinearizing step: the fused linearize + point stage
    # (ms_linearize), then the pair and diagonal stages (ms_form_rcs)
    rl = [k for k in range(args.steps) if relin[k]]
    if not rl:
        raise RuntimeError("no timed step relinearized; raise --steps")
    t_form = float(np.mean([infos[k]["ms_linearize"] + infos[k]["ms_form_rcs"] for k in rl]))
    value = scene.n_obs / (t_form * 1e-3)
    st_arr = np.array(stages)
    stage_ms = {"linpoint": float(np.mean([st_arr[k, 0] for k in rl])),
                "pair": float(np.mean([st_arr[k, 2] for k in rl])),
                "diag": float(np.mean([st_arr[k, 3] for k in rl]))}
    alg = stage_bytes(scene, sizes, args.precision)
    wl_key = f"{args.workload}_{args.precision}"
    stages_roof = {}
    for name in ("linpoint", "pair", "diag"):
        kern = KERNEL_OF_STAGE[name][args.precision]
        stages_roof[name] = roofline_entry(kern, alg[name], stage_ms[name],
                                           traffic_from_profile(f"{kern}_{wl_key}"))
    dominant = max(stage_ms, key=stage_ms.get)
    total_alg = sum(alg.values())
    form_roof = roofline_entry("k_linpoint + k_offdiag + k_diag (whole formation)", total_alg, t_form, None)
    form_roof["bytes_per_obs"] = total_alg / scene.n_obs
    out = {
        "metric": METRIC, "value": value, "unit": "obs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32/f64",
        "data": "synthetic",
        "config": {"workload": f"{scene.name} ({scene.n_obs} observations, {int(scene.cam_fixed.sum())} fixed "
                               f"cameras), {'FP64' if args.precision == 'fp64' else 'mixed FP32/FP64'}, "
                               f"{args.precond.replace('_', '-')}{' + gauge-deflated' if args.deflate else ''}"
                               f"{' (FP32 solver matrix)' if args.solver_fp32 else ''} "
                               f"PCG to rel {scene.pcg_tol:g}",
                   "n_cams": scene.n_cams, "n_pts": scene.n_pts, "n_obs": scene.n_obs,
                   "n_rows": sizes["n_rows"], "n_blocks": sizes["n_blk"], "n_pairs": sizes["n_pairs"],
                   "pcg_product": args.product},
        "lm_iteration_ms": ms_per_step,
        "formation_ms": t_form,
        "create_ms": create_ms,
        "formation_steps_counted": len(rl),
        "stages_ms": {**stage_ms,
                      "reformation_after_rejection": float(np.mean([infos[k]["ms_form_rcs"] for k in range(args.steps)
                                                                    if not relin[k]]))
                      if len(rl) < args.steps else None,
                      "pcg": float(np.mean([i["ms_pcg"] for i in infos])),
                      "back_substitute": float(np.mean([i["ms_back_substitute"] for i in infos])),
                      "evaluate": float(np.mean([i["ms_evaluate"] for i in infos]))},
        "pcg_iters": [int(i["pcg_iters"]) for i in infos],
        "pcg_relres": [float(i["pcg_relres"]) for i in infos],
        "pcg_capped": int(sum(i["pcg_status"] == ba.BA_ERR_NOT_CONVERGED for i in infos)),
        "final_cost": float(min(i["cost_new"] if i["accepted"] else i["cost"] for i in infos)),
        "roofline": stages_roof[dominant],
        "stages_roofline": stages_roof,
        "formation_roofline": form_roof,
    }
    out["bsmc_vs_csr"] = storage_comparison(ctx, sizes["n_rows"], dev)
    cp = copy_peak_gbs(dev)
    for ent in list(stages_roof.values()) + [form_roof]:
        ent["copy_peak"] = cp
        ent["frac_of_copy_peak"] = ent["achieved"] / cp
    if net is not None:
        ba.ba_set_preconditioner_net(ctx, None)
        ba.ba_gnn_destroy(net)
    ba.ba_destroy(ctx)
    torch.cuda.empty_cache()
    if not args.no_compare:
        names = ([v[0] for v in COMPARE_VARIANTS] if args.compare == "all" else
                 DEFAULT_VARIANTS if args.compare == "default" else args.compare.split(","))
        obs = (obs_cam, obs_pt, uv, cf)
        out["lm_comparison"] = lm_comparison(scene, obs, names, args.lm_iters or scene.lm_iterations,
                                             PRODUCTS[args.product])
        if args.aerial_compare and args.workload != "aerial":
            ascene = build_scene("aerial")
            aobs = device_observations(ascene, dev)
            out["lm_comparison_aerial"] = lm_comparison(ascene, aobs, names, ascene.lm_iterations,
                                                        PRODUCTS[args.product])
            del aobs
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        progress(f"oracle on {args.cpu_sample}")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample, args.cpu_lm_iters, scene.n_obs)
        out["cpu_baseline"]["gpu_lm_iteration_ms_per_obs"] = ms_per_step / scene.n_obs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
