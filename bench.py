"""Benchmark of the bundle-adjustment hot path on one MI355X.

A step is one LM iteration (linearize, RCS formation, block-Jacobi PCG to
rel 1e-6, back-substitution, candidate cost and gain ratio) on the aerial
grid scene: 2,000 nadir cameras on a 50 x 40 grid, 400,000 points, track
length truncated-geometric on [2, 12] with mean 4 (~1.6M observations),
pixel noise N(0, 0.5^2), FP64.  Inputs are synthetic and resident in HBM
before timing starts.

Printed JSON line: value = RCS formation throughput (observations per
second through linearize + formation, device time of the timed steps);
ms_per_step = LM-iteration wall time; the roofline entry covers the
dominant formation kernel (the camera-pair stage); cpu_baseline is the C
oracle on the host cores for a bounded sample of the same workload.
lm_comparison: LM runs of the preconditioner / precision variants on the
same scene; lm_comparison_partition: the key variants on the one-GPU share
of the 60,000-camera partition (25M points, ~100M observations, mixed
precision and the learned preconditioner against plain FP64 block-Jacobi,
10 LM iterations).
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
    ap.add_argument("--workload", default="aerial", choices=["aerial", "strips", "partition"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-formations", type=int, default=2)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the learned + mixed vs FP64 block-Jacobi LM comparison")
    ap.add_argument("--lm-iters", type=int, default=None,
                    help="LM iterations of each compared run (default: the workload's budget)")
    ap.add_argument("--compare", default="all",
                    help="comma-separated subset of the compared runs, or 'all'")
    ap.add_argument("--precond", default="block_jacobi",
                    choices=["block_jacobi", "fsai", "learned", "learned_fsai"],
                    help="preconditioner of the timed LM steps")
    ap.add_argument("--deflate", action="store_true", help="gauge-deflated PCG in the timed LM steps")
    ap.add_argument("--no-partition-compare", action="store_true",
                    help="skip the LM comparison on the 60,000-camera partition after the default run")
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
    return scenegen.partition_scene(seed=2, with_stats=False)


def pair_stage_bytes(n_pairs, n_offseg, precision):
    """Algorithmic bytes of one camera-pair-stage launch: per observation
    couple its two index words and the two 24-value records (J_c and K), per
    off-diagonal block its 81 FP64 outputs and its segment bounds."""
    es = 4 if precision == "mixed" else 8
    return n_pairs * (8 + 2 * 24 * es) + n_offseg * (81 * 8 + 8)


def traffic_from_profile(kernel_src_hash, kernel):
    """HBM traffic per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        ent = d.get(kernel)
        if ent and ent.get("source_sha256") == kernel_src_hash:
            return ent.get("bytes_per_launch")
    except Exception:
        return None
    return None


def lm_run(scene, obs, precision, precond, iters, learned_weights=None, deflate=False, solver_fp32=False,
           product=0):
    """LM run from the scene's start; returns per-iteration means and the
    final cost (FP64 cost of the last accepted iterate)."""
    import torch
    from paper_2307_08383_amd import ba
    obs_cam, obs_pt, uv, cf = obs
    ctx = ba.ba_create(scene.n_cams, scene.n_pts, obs_cam, obs_pt, uv, cf, precision=precision)
    net = None
    if precond in (ba.BA_PRECOND_LEARNED, ba.BA_PRECOND_LEARNED_FSAI):
        net = ba.ba_gnn_create(learned_weights)
        ba.ba_set_preconditioner_net(ctx, net)
    dev = uv.device
    cams = torch.as_tensor(scene.cams_init, dtype=torch.float64, device=dev).contiguous()
    pts = torch.as_tensor(scene.pts_init, dtype=torch.float64, device=dev).contiguous()
    # one-time structures built on first use (index sets of the FSAI pattern,
    # the network's graph, the FP32 copy), like the co-visibility pattern at
    # creation: built here, outside the timed run, from a formed RCS at the
    # start point (parameters unchanged), and reported separately
    setup_ms = 0.0
    if precond != ba.BA_PRECOND_BLOCK_JACOBI or deflate or solver_fp32:
        torch.cuda.synchronize()
        t_s = time.perf_counter()
        ba.ba_linearize(ctx, cams, pts)
        ba.ba_form_rcs(ctx, 1e-4)
        dx = torch.empty((ba.ba_get_sizes(ctx)["n_rows"], 9), dtype=torch.float64, device=dev)
        ba.ba_pcg_solve(ctx, dx, tol=scene.pcg_tol, max_iter=1, precond=precond, deflate=deflate,
                        solver_fp32=solver_fp32, product=product)
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t_s)
    st = ba.new_lm_state(1e-4)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
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
    return dict(ms_per_iter=1e3 * wall / iters, final_cost=final, first_use_setup_ms=setup_ms,
                accepted=int(sum(i["accepted"] for i in infos)),
                pcg_iters=[int(i["pcg_iters"]) for i in infos],
                pcg_iters_mean=float(np.mean([i["pcg_iters"] for i in infos])),
                precond_ms_mean=float(np.mean([i["ms_precond"] for i in infos])),
                form_ms_mean=float(np.mean([i["ms_form_rcs"] for i in infos])),
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
    ("mixed_block_jacobi_deflated", "mixed", "block_jacobi", True),
    ("mixed_fsai", "mixed", "fsai", False),
    ("mixed_fsai_deflated", "mixed", "fsai", True),
    ("mixed_learned_block_deflated", "mixed", "learned", True),
    ("mixed_learned_fsai", "mixed", "learned_fsai", False),
    ("mixed_learned_fsai_deflated", "mixed", "learned_fsai", True),
    ("mixed_s32_block_jacobi_deflated", "mixed", "block_jacobi", True),
    ("mixed_s32_fsai_deflated", "mixed", "fsai", True),
    ("mixed_s32_learned_fsai_deflated", "mixed", "learned_fsai", True)]
# the subset run on the 60,000-camera partition (the one-GPU share the
# learned-vs-block-Jacobi comparison is defined on) after the default run
PARTITION_VARIANTS = ["fp64_block_jacobi", "mixed_block_jacobi_deflated", "mixed_fsai_deflated",
                      "mixed_learned_fsai_deflated", "mixed_s32_block_jacobi_deflated",
                      "mixed_s32_learned_fsai_deflated"]


def lm_comparison(scene, obs, names, lm_iters, product=0):
    """Each named variant from the scene's start for lm_iters LM iterations;
    ms per iteration, final FP64 cost and the ratios to FP64 block-Jacobi."""
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
        progress(f"LM comparison {scene.name} {name}: {runs[name]['ms_per_iter']:.2f} ms per iteration")
    base = runs["fp64_block_jacobi"]
    return {
        "scene": scene.name, "n_obs": scene.n_obs, "iterations": lm_iters,
        **runs,
        "learned_weights": {"block": wb_name, "fsai": wf_name},
        "speedup_vs_fp64_block_jacobi": {k: base["ms_per_iter"] / v["ms_per_iter"] for k, v in runs.items()},
        "final_cost_rel_diff_vs_fp64_block_jacobi": {
            k: abs(v["final_cost"] - base["final_cost"]) / base["final_cost"] for k, v in runs.items()},
    }


def formation_roofline(scene, sizes, precision, t_form_ms):
    """Algorithmic HBM bytes of one formation (linearize + point stage, pair
    stage, diagonal stage; the per-unit counts of the kernels' design) over
    its device time."""
    es = 4 if precision == "mixed" else 8
    n, npt = scene.n_obs, scene.n_pts
    free_obs = int((~scene.cam_fixed.astype(bool))[scene.obs_cam].sum())
    lin = n * (28 + 24 * es + 6 * es + 16 + 16) + npt * (24 + 72)
    pair = pair_stage_bytes(sizes["n_pairs"], sizes["n_blk"] - sizes["n_rows"], precision)
    diag = free_obs * (24 * es + 16 + 4) + sizes["n_rows"] * 1368
    total = lin + pair + diag
    achieved = total / (t_form_ms * 1e-3) / 1e9
    return {"bound": "hbm", "bytes_per_obs": total / n, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "stages": {"linearize_point": lin, "pair": pair, "diag": diag}}


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


def cpu_baseline(scene, n_form):
    from oracle import oracle as orc
    nt = orc.default_threads()
    uv = orc.observations(scene)
    P = orc.Problem.from_scene(scene, uv, n_threads=nt)
    t0 = time.perf_counter()
    for _ in range(n_form):
        P.linearize(scene.cams_init, scene.pts_init)
        P.form_rcs(1e-4)
    dt = time.perf_counter() - t0
    # one thread, one formation
    P1 = orc.Problem.from_scene(scene, uv, n_threads=1)
    t1 = time.perf_counter()
    P1.linearize(scene.cams_init, scene.pts_init)
    P1.form_rcs(1e-4)
    dt1 = time.perf_counter() - t1
    return {"value": scene.n_obs * n_form / dt, "unit": "obs/s", "cores": nt, "kind": "oracle",
            "sample": f"the full scene ({scene.n_obs} observations), {n_form} formations "
                      f"(linearize + RCS formation), {dt:.2f} s",
            "single_thread_value": scene.n_obs / dt1, "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


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
    ctx = ba.ba_create(scene.n_cams, scene.n_pts, obs_cam, obs_pt, uv, cf, precision=prec)
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
    infos, stages = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(ba.ba_lm_step(ctx, cams, pts, st, **step_kw))
        stages.append(ba.ba_get_stage_ms(ctx))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    lin = [i["ms_linearize"] for i in infos if i["ms_linearize"] > 0]
    form = [i["ms_form_rcs"] for i in infos]
    t_form = (np.mean(lin) if lin else 0.0) + np.mean(form)
    value = scene.n_obs / (t_form * 1e-3)
    st_arr = np.array(stages)
    pair_ms = float(st_arr[:, 2].mean())
    n_offseg = sizes["n_blk"] - sizes["n_rows"]
    alg = pair_stage_bytes(sizes["n_pairs"], n_offseg, args.precision)
    achieved = alg / (pair_ms * 1e-3) / 1e9
    src = open(os.path.join(ROOT, "paper_2307_08383_amd", "csrc", "kernels_rcs.hip"), "rb").read()
    traffic = traffic_from_profile(hashlib.sha256(src).hexdigest(),
                                   f"k_offdiag_{args.workload}_{args.precision}")
    out = {
        "metric": METRIC, "value": value, "unit": "obs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32/f64",
        "data": "synthetic",
        "config": {"workload": f"{scene.name} ({scene.n_obs} observations), "
                               f"{'FP64' if args.precision == 'fp64' else 'mixed FP32/FP64'}, "
                               f"{args.precond.replace('_', '-')}{' + gauge-deflated' if args.deflate else ''}"
                               f"{' (FP32 solver matrix)' if args.solver_fp32 else ''} "
                               f"PCG to rel {scene.pcg_tol:g}",
                   "n_cams": scene.n_cams, "n_pts": scene.n_pts, "n_obs": scene.n_obs,
                   "n_blocks": sizes["n_blk"], "n_pairs": sizes["n_pairs"], "pcg_product": args.product},
        "lm_iteration_ms": ms_per_step,
        "formation_ms": t_form,
        "stages_ms": {"linearize": float(st_arr[:, 0][st_arr[:, 0] > 0].mean()) if (st_arr[:, 0] > 0).any() else 0.0,
                      "point": float(st_arr[:, 1].mean()), "pair": pair_ms, "diag": float(st_arr[:, 3].mean()),
                      "pcg": float(np.mean([i["ms_pcg"] for i in infos])),
                      "back_substitute": float(np.mean([i["ms_back_substitute"] for i in infos])),
                      "evaluate": float(np.mean([i["ms_evaluate"] for i in infos]))},
        "pcg_iters_mean": float(np.mean([i["pcg_iters"] for i in infos])),
        "final_cost": float(min(i["cost_new"] if i["accepted"] else i["cost"] for i in infos)),
        "roofline": {"kernel": "k_offdiag (camera-pair stage)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": alg},
        "formation_roofline": formation_roofline(scene, sizes, args.precision, t_form),
    }
    cp = copy_peak_gbs(dev)
    out["roofline"]["copy_peak"] = cp
    out["roofline"]["frac_of_copy_peak"] = achieved / cp
    out["formation_roofline"]["frac_of_copy_peak"] = out["formation_roofline"]["achieved"] / cp
    if net is not None:
        ba.ba_set_preconditioner_net(ctx, None)
        ba.ba_gnn_destroy(net)
    ba.ba_destroy(ctx)
    if not args.no_compare:
        names = [v[0] for v in COMPARE_VARIANTS] if args.compare == "all" else args.compare.split(",")
        obs = (obs_cam, obs_pt, uv, cf)
        out["lm_comparison"] = lm_comparison(scene, obs, names, args.lm_iters or scene.lm_iterations,
                                             PRODUCTS[args.product])
        if args.workload != "partition" and not args.no_partition_compare:
            pscene = build_scene("partition")
            progress(f"scene {pscene.name}: {pscene.n_obs} observations")
            pobs = device_observations(pscene, dev)
            out["lm_comparison_partition"] = lm_comparison(pscene, pobs, PARTITION_VARIANTS, pscene.lm_iterations,
                                                           PRODUCTS[args.product])
            del pobs
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, args.cpu_sample_formations)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
