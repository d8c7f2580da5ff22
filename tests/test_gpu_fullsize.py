"""Full-size parity (needs a GPU): the aerial scene (2,000 cameras, 1.6M
observations) in FP64, the strip scene (20,000 cameras, ~20M observations)
in mixed precision and the partition scene (60,000 free cameras plus a ring
of fixed ones, ~100M observations) in both precisions, against the oracle
on the same inputs; on the two large scenes also the PCG product S x in
both layouts.  LM runs: 20 iterations on the aerial scene against the
oracle's run (both precisions, with the per-iteration cost error and the
error of the first step's dx reported), 10 iterations on the strip scene
(both precisions) and on the partition against the oracle's stored runs.
Each report is printed, and also saved as JSON in the repository's output
folder when that folder exists."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2307_08383_amd import scenegen

from gpu_util import T, block_errors, create

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
ba = pytest.importorskip("paper_2307_08383_amd.ba")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _report(name, d):
    out = os.path.join(ROOT, "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, name), "w") as f:
            json.dump(d, f, indent=1)
    print(name, json.dumps(d), flush=True)


def _block_product(blk, rp, ci, x):
    """y = S x from the upper blocks (both triangles), and |S| |x|."""
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    y = np.zeros_like(x)
    a = np.zeros_like(x)
    np.add.at(y, rows, np.einsum("kij,kj->ki", blk, x[ci]))
    np.add.at(a, rows, np.einsum("kij,kj->ki", np.abs(blk), np.abs(x[ci])))
    off = ci != rows
    np.add.at(y, ci[off], np.einsum("kji,kj->ki", blk[off], x[rows[off]]))
    np.add.at(a, ci[off], np.einsum("kji,kj->ki", np.abs(blk[off]), np.abs(x[rows[off]])))
    return y, a


def _rcs_case(scene, precision, lam=1e-4, products=None):
    """Per-block RCS errors against the oracle; with `products` (a dict) also
    y = S x in both PCG product layouts for one random x, checked against
    the product of the stored blocks and of the oracle's blocks."""
    uv = orc.observations(scene)
    P = orc.Problem.from_scene(scene, uv)
    P.linearize(scene.cams_init, scene.pts_init)
    P.form_rcs(lam)
    ctx = create(scene, uv, precision)
    ys = {}
    try:
        ba.ba_linearize(ctx, T(scene.cams_init, torch.float64), T(scene.pts_init, torch.float64))
        ba.ba_form_rcs(ctx, lam)
        rp, ci = ba.ba_get_pattern(ctx)
        rp_ref, ci_ref = P.pattern()
        assert np.array_equal(rp, rp_ref) and np.array_equal(ci, ci_ref)
        blk, rhs = ba.ba_get_rcs(ctx)
        if products is not None:
            x = np.random.default_rng(5).standard_normal((len(rp) - 1, 9))
            xd = T(x, torch.float64)
            for prod in (ba.BA_PRODUCT_FULL, ba.BA_PRODUCT_UPPER):
                y = torch.empty_like(xd)
                ba.ba_rcs_product(ctx, xd, y, product=prod)
                ys[prod] = y.cpu().numpy()
    finally:
        ba.ba_destroy(ctx)
    blk_ref, rhs_ref = P.rcs()
    errs, raw = block_errors(blk, blk_ref, rp_ref, ci_ref)
    rerr = np.linalg.norm(rhs - rhs_ref, axis=1) / np.linalg.norm(rhs_ref, axis=1)
    if products is not None:
        y_own, a_own = _block_product(blk, rp, ci, x)
        y_ref, a_ref = _block_product(blk_ref, rp_ref, ci_ref, x)
        for prod, name in ((ba.BA_PRODUCT_FULL, "full"), (ba.BA_PRODUCT_UPPER, "upper")):
            products[f"{name}_vs_stored_blocks"] = float(np.max(np.abs(ys[prod] - y_own) / a_own))
            products[f"{name}_vs_oracle_blocks"] = float(np.max(np.abs(ys[prod] - y_ref) / a_ref))
    return errs, raw, rerr


@pytest.mark.timeout(600)
def test_benchmark_scene_fp64_rcs():
    s = scenegen.aerial_grid_scene(seed=0, with_stats=False)
    errs, raw, rerr = _rcs_case(s, 0)
    rep = dict(scene=s.name, n_obs=s.n_obs, n_blocks=len(errs), max_block_err=float(errs.max()),
               p999_block_err=float(np.quantile(errs, 0.999)), max_raw_rel=float(raw.max()),
               max_rhs_rel=float(rerr.max()))
    _report("fullsize_fp64_rcs.json", rep)
    assert errs.max() <= 1e-10 and rerr.max() <= 1e-9


@pytest.mark.timeout(900)
def test_strip_scene_mixed_rcs_errors():
    s = scenegen.strips_scene(seed=1, with_stats=False)
    prods = {}
    errs, raw, rerr = _rcs_case(s, 1, products=prods)
    rep = dict(scene=s.name, n_obs=s.n_obs, n_blocks=len(errs), max_block_err=float(errs.max()),
               p999_block_err=float(np.quantile(errs, 0.999)), median_block_err=float(np.median(errs)),
               max_raw_rel=float(raw.max()), p999_raw_rel=float(np.quantile(raw, 0.999)),
               max_rhs_rel=float(rerr.max()), p999_rhs_rel=float(np.quantile(rerr, 0.999)), products=prods)
    _report("fullsize_mixed_rcs_errors.json", rep)
    assert errs.max() <= 1e-4
    _check_products(prods)


def _check_products(prods):
    """Both layouts form S x of the stored blocks up to summation order, and
    match the oracle's S within the per-block tolerance of the mixed path."""
    for name in ("full", "upper"):
        assert prods[f"{name}_vs_stored_blocks"] <= 1e-13
        assert prods[f"{name}_vs_oracle_blocks"] <= 1e-4


@pytest.mark.timeout(900)
def test_benchmark_scene_lm_final_cost():
    """20 LM iterations (the benchmark configuration): final cost of the
    FP64 path and of the mixed path against the oracle, rel 1e-6."""
    s = scenegen.aerial_grid_scene(seed=0, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    c_ref, p_ref, hist_ref = orc.lm_run(P, s.cams_init, s.pts_init, 20)
    F_ref = P.cost(c_ref, p_ref)
    rep = dict(scene=s.name, oracle_final_cost=F_ref)
    # the first step's dx at lambda 1e-4 (PCG to rel 1e-12; the RCS is
    # ill-conditioned along the similarity gauge, so this is an error report,
    # bounded only loosely)
    P.linearize(s.cams_init, s.pts_init)
    P.form_rcs(1e-4)
    xc_ref, _ = P.pcg(tol=1e-12, max_iter=20000)
    xp_ref = P.back_substitute(xc_ref)
    for precision in (0, 1):
        tag = "fp64" if precision == 0 else "mixed"
        ctx = create(s, uv, precision)
        try:
            cams = T(s.cams_init, torch.float64)
            pts = T(s.pts_init, torch.float64)
            ba.ba_linearize(ctx, cams, pts)
            ba.ba_form_rcs(ctx, 1e-4)
            xc = torch.empty((P.n_rows, 9), dtype=torch.float64, device="cuda")
            xp = torch.empty((s.n_pts, 3), dtype=torch.float64, device="cuda")
            ba.ba_pcg_solve(ctx, xc, tol=1e-12, max_iter=20000)
            ba.ba_back_substitute(ctx, xc, xp)
            rep[f"dx_cam_rel_err_{tag}"] = float(np.linalg.norm(xc.cpu().numpy() - xc_ref) / np.linalg.norm(xc_ref))
            rep[f"dx_pt_rel_err_{tag}"] = float(np.linalg.norm(xp.cpu().numpy() - xp_ref) / np.linalg.norm(xp_ref))
            st = ba.new_lm_state(1e-4)
            hist = [ba.ba_lm_step(ctx, cams, pts, st) for _ in range(20)]
            F = P.cost(cams.cpu().numpy(), pts.cpu().numpy())
        finally:
            ba.ba_destroy(ctx)
        rep[f"final_cost_{tag}"] = F
        rep[f"rel_diff_{tag}"] = abs(F - F_ref) / F_ref
        rep[f"cost_rel_err_per_iteration_{tag}"] = [abs(h["cost"] - r["cost"]) / r["cost"]
                                                     for h, r in zip(hist, hist_ref)]
        rep[f"accepted_{tag}"] = [h["accepted"] for h in hist]
    rep["oracle_accepted"] = [r["accepted"] for r in hist_ref]
    _report("fullsize_lm_final_cost.json", rep)
    assert rep["rel_diff_fp64"] <= 1e-6 and rep["rel_diff_mixed"] <= 1e-6
    assert rep["dx_cam_rel_err_fp64"] <= 1e-3 and rep["dx_cam_rel_err_mixed"] <= 1e-1


@pytest.fixture(scope="module")
def partition_case():
    """The 60,000-camera partition (seed 2) with the oracle's FP64 RCS at the
    start, lambda 1e-4; the oracle problem is kept to evaluate costs."""
    s = scenegen.partition_scene(seed=2, with_stats=False)
    uv = orc.observations(s)
    P = orc.Problem.from_scene(s, uv)
    P.linearize(s.cams_init, s.pts_init)
    P.form_rcs(1e-4)
    blk_ref, rhs_ref = P.rcs()
    rp_ref, ci_ref = P.pattern()
    return s, uv, P, blk_ref, rhs_ref, rp_ref, ci_ref


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("precision", [0, 1])
def test_partition_scene_rcs(partition_case, precision):
    """Both precisions against the same oracle RCS: per-block error 1e-10
    (FP64) / 1e-4 (mixed), pattern bit-exact; the mixed run also checks the
    PCG product in both layouts."""
    s, uv, P, blk_ref, rhs_ref, rp_ref, ci_ref = partition_case
    ctx = create(s, uv, precision)
    prods = {} if precision == 1 else None
    try:
        ba.ba_linearize(ctx, T(s.cams_init, torch.float64), T(s.pts_init, torch.float64))
        ba.ba_form_rcs(ctx, 1e-4)
        rp, ci = ba.ba_get_pattern(ctx)
        assert np.array_equal(rp, rp_ref) and np.array_equal(ci, ci_ref)
        blk, rhs = ba.ba_get_rcs(ctx)
        x = np.random.default_rng(5).standard_normal((len(rp) - 1, 9))
        xd = T(x, torch.float64)
        ys = {}
        # mixed: the two PCG layouts; FP64: the CSR copy (Eq. (8) storage)
        for prod in ((ba.BA_PRODUCT_FULL, ba.BA_PRODUCT_UPPER) if prods is not None else (ba.BA_PRODUCT_CSR,)):
            y = torch.empty_like(xd)
            ba.ba_rcs_product(ctx, xd, y, product=prod)
            ys[prod] = y.cpu().numpy()
    finally:
        ba.ba_destroy(ctx)
    errs, raw = block_errors(blk, blk_ref, rp_ref, ci_ref)
    rerr = np.linalg.norm(rhs - rhs_ref, axis=1) / np.linalg.norm(rhs_ref, axis=1)
    del blk
    rep = dict(scene=s.name, precision="fp64" if precision == 0 else "mixed", n_obs=s.n_obs,
               n_fixed=int(s.cam_fixed.sum()), n_blocks=len(errs),
               max_block_err=float(errs.max()), p999_block_err=float(np.quantile(errs, 0.999)),
               median_block_err=float(np.median(errs)), max_raw_rel=float(raw.max()),
               p999_raw_rel=float(np.quantile(raw, 0.999)), max_rhs_rel=float(rerr.max()),
               p999_rhs_rel=float(np.quantile(rerr, 0.999)))
    y_ref, a_ref = _block_product(blk_ref, rp_ref, ci_ref, x)
    if prods is None:
        rep["csr_product_vs_oracle_blocks"] = float(np.max(np.abs(ys[ba.BA_PRODUCT_CSR] - y_ref) / a_ref))
    else:
        for prod, name in ((ba.BA_PRODUCT_FULL, "full"), (ba.BA_PRODUCT_UPPER, "upper")):
            prods[f"{name}_vs_oracle_blocks"] = float(np.max(np.abs(ys[prod] - y_ref) / a_ref))
        prods["full_vs_upper"] = float(np.max(np.abs(ys[ba.BA_PRODUCT_FULL] - ys[ba.BA_PRODUCT_UPPER]) / a_ref))
        rep["products"] = prods
    _report(f"fullsize_partition_{rep['precision']}_rcs_errors.json", rep)
    if precision == 0:
        assert errs.max() <= 1e-10 and rerr.max() <= 1e-9
        assert rep["csr_product_vs_oracle_blocks"] <= 1e-10
    else:
        assert errs.max() <= 1e-4
        for name in ("full", "upper"):
            assert prods[f"{name}_vs_oracle_blocks"] <= 1e-4
        assert prods["full_vs_upper"] <= 1e-13


GOLDEN_LM = os.path.join(ROOT, "tests", "golden", "partition60000_lm_oracle.json")
GOLDEN_STRIPS_LM = os.path.join(ROOT, "tests", "golden", "strips20000_lm_oracle.json")


def _lm_against_oracle_run(s, uv, P, golden, precision, precond, deflate, weights=None):
    """The library's LM run of the stored run's budget from the start (PCG
    tolerance and cap as stored, else the scene's and 1000); per-step
    records and the oracle's cost of the final parameters."""
    ctx = create(s, uv, precision)
    net = None
    try:
        if weights is not None:
            net = ba.ba_gnn_create(weights)
            ba.ba_set_preconditioner_net(ctx, net)
        cams = T(s.cams_init, torch.float64)
        pts = T(s.pts_init, torch.float64)
        st = ba.new_lm_state(1e-4)
        hist = []
        for _ in range(len(golden["iterations"])):
            lam0 = st.lam
            h = ba.ba_lm_step(ctx, cams, pts, st, pcg_tol=golden.get("pcg_tol", s.pcg_tol),
                              pcg_max_iter=golden.get("pcg_max_iter", 1000), precond=precond, deflate=deflate)
            h["lambda_before"] = lam0
            hist.append(h)
        F = P.cost(cams.cpu().numpy(), pts.cpu().numpy())
    finally:
        if net is not None:
            ba.ba_set_preconditioner_net(ctx, None)
            ba.ba_gnn_destroy(net)
        ba.ba_destroy(ctx)
    return hist, F


@pytest.mark.timeout(900)
def test_strip_scene_lm_against_oracle_run():
    """10 LM iterations on the strip scene (20,000 cameras, ~20M
    observations: the scene the mixed-precision path is reported on) against
    the oracle's own run of the same budget (stored by
    tests/golden/make_strips_lm.py from the oracle alone).  This start is far
    from the optimum (the first step lowers F about 200-fold, the second
    overshoots and is rejected), so the run is compared where it is
    reproducible: every step solved to rel 1e-12 as in the stored run, with
    a cap no step reaches.  FP64: every decision, the cost entering each of
    the 10 iterations (so every accepted step's F' but the last) and the
    rejected step's F' to rel 1e-6.  The tenth step is not reproducible: from
    iterates whose costs agree to 5e-7 and with both solves converged to rel
    1e-12, its F' differed by 3.5e-4 (the step is long and the system
    ill-conditioned: solutions with equal residuals differ along the
    smallest eigenvectors, and this start's F' depends on them), so the last
    F' and the final cost are reported.  Mixed precision: its steps differ
    from FP64's by the FP32 rounding of the records (block errors up to
    about 3e-7 here), which the rejected second step amplifies to 1e-2, so
    its first step is held to rel 1e-6 (measured 1e-7) and the rest of its
    run is reported against the oracle's."""
    import hashlib
    s = scenegen.strips_scene(seed=1, with_stats=False)
    uv = orc.observations(s)
    golden = json.load(open(GOLDEN_STRIPS_LM))
    assert golden["scene_digest"] == s.digest()
    assert golden["uv_sha256"] == hashlib.sha256(np.ascontiguousarray(uv).tobytes()).hexdigest()
    P = orc.Problem.from_scene(s, uv)
    ref = golden["iterations"]
    F_ref = golden["final_cost"]
    rep = dict(scene=s.name, pcg_tol=golden["pcg_tol"], oracle_final_cost=F_ref, oracle_iterations=[
        dict(cost=r["cost"], cost_new=r["cost_new"], accepted=r["accepted"], pcg_iters=r["pcg_iters"])
        for r in ref])
    for name, precision in (("fp64_block_jacobi", 0), ("mixed_block_jacobi", 1)):
        hist, F = _lm_against_oracle_run(s, uv, P, golden, precision, ba.BA_PRECOND_BLOCK_JACOBI, False)
        per_it = [dict(cost_rel_err=abs(h["cost"] - r["cost"]) / r["cost"],
                       cost_new_rel_err=abs(h["cost_new"] - r["cost_new"]) / r["cost_new"],
                       accepted=h["accepted"], oracle_accepted=r["accepted"], pcg_iters=h["pcg_iters"],
                       pcg_relres=h["pcg_relres"]) for h, r in zip(hist, ref)]
        rep[name] = dict(final_cost=F, final_cost_rel_diff=abs(F - F_ref) / F_ref, iterations=per_it)
    _report("fullsize_strips_lm_vs_oracle.json", rep)
    d = rep["fp64_block_jacobi"]
    assert len(d["iterations"]) == len(ref)
    for it, r in zip(d["iterations"], ref):
        assert it["cost_rel_err"] <= 1e-6, it
        assert it["pcg_relres"] <= 1e-12, it
        if abs(r["cost"] - r["cost_new"]) > 1e-8 * r["cost"]:
            assert it["accepted"] == r["accepted"]
            if not r["accepted"]:
                assert it["cost_new_rel_err"] <= 1e-6, it
    m = rep["mixed_block_jacobi"]["iterations"][0]
    assert m["cost_rel_err"] <= 1e-12 and m["accepted"] == ref[0]["accepted"]
    assert m["cost_new_rel_err"] <= 1e-6, m


@pytest.mark.timeout(1200)
def test_partition_lm_against_oracle_run(partition_case):
    """10 LM iterations on the partition (the configuration the learned vs
    block-Jacobi comparison is defined on) against the oracle's own run of
    the same budget (stored by tests/golden/make_partition_lm.py from the
    oracle alone): FP64 block-Jacobi, and mixed precision with the learned
    factorised preconditioner and gauge deflation.  Decisions are compared
    where the oracle's step is far from a tie and the final cost at rel 1e-6.
    FP64 block-Jacobi runs the oracle's algorithm, so its cost at every
    iteration is held to rel 1e-6 too; the mixed learned variant solves each
    step's system with another preconditioner in another precision, so its
    step equals the oracle's only to the PCG tolerance (rel 1e-6 residual),
    which on the first steps, far from the optimum, moves F' by up to about
    1e-5 relative (bound 2e-5 per iteration)."""
    import hashlib
    from paper_2307_08383_amd import learned_precond as lp
    s, uv, P, _, _, _, _ = partition_case
    golden = json.load(open(GOLDEN_LM))
    assert golden["scene_digest"] == s.digest()
    assert golden["uv_sha256"] == hashlib.sha256(np.ascontiguousarray(uv).tobytes()).hexdigest()
    ref = golden["iterations"]
    F_ref = golden["final_cost"]
    variants = [("fp64_block_jacobi", 0, ba.BA_PRECOND_BLOCK_JACOBI, False, None),
                ("mixed_learned_fsai_deflated", 1, ba.BA_PRECOND_LEARNED_FSAI, True,
                 lp.load_weights(lp.DEFAULT_FSAI_WEIGHTS))]
    rep = dict(scene=s.name, oracle_final_cost=F_ref, oracle_iterations=[
        dict(cost=r["cost"], cost_new=r["cost_new"], accepted=r["accepted"], pcg_iters=r["pcg_iters"])
        for r in ref])
    for name, precision, pre, defl, w in variants:
        hist, F = _lm_against_oracle_run(s, uv, P, golden, precision, pre, defl, w)
        per_it = []
        for h, r in zip(hist, ref):
            per_it.append(dict(cost_rel_err=abs(h["cost"] - r["cost"]) / r["cost"],
                               cost_new_rel_err=abs(h["cost_new"] - r["cost_new"]) / r["cost_new"],
                               accepted=h["accepted"], oracle_accepted=r["accepted"],
                               pcg_iters=h["pcg_iters"], pcg_relres=h["pcg_relres"],
                               precond_fallback=h["precond_fallback"]))
        rep[name] = dict(final_cost=F, final_cost_rel_diff=abs(F - F_ref) / F_ref, iterations=per_it)
    _report("fullsize_partition_lm_vs_oracle.json", rep)
    for name, precision, _, _, _ in variants:
        d = rep[name]
        assert d["final_cost_rel_diff"] <= 1e-6, (name, d["final_cost_rel_diff"])
        bound = 1e-6 if name == "fp64_block_jacobi" else 2e-5
        for it, r in zip(d["iterations"], ref):
            if abs(r["cost"] - r["cost_new"]) > 1e-8 * r["cost"]:
                assert it["accepted"] == r["accepted"], name
                assert it["cost_rel_err"] <= bound, (name, it)


@pytest.mark.timeout(600)
def test_partition_triangulation_sampled(partition_case):
    """Re-triangulation of all 25M points of the partition on the GPU (linear
    start + 4 Gauss-Newton steps, the cameras at the start) against the
    oracle on every 997th point."""
    s, uv, P, _, _, _, _ = partition_case
    which = np.arange(0, s.n_pts, 997, dtype=np.int32)
    X_ref, nf_ref = P.triangulate(s.cams_init, s.pts_init, init=True, n_gn=4, which=which)
    ctx = create(s, uv, 0)
    try:
        pts = T(s.pts_init, torch.float64)
        nf = ba.ba_triangulate(ctx, T(s.cams_init, torch.float64), pts, linear_init=True, n_gn=4)
        X = pts[torch.as_tensor(which, device=pts.device, dtype=torch.int64)].cpu().numpy()
    finally:
        ba.ba_destroy(ctx)
    err = np.abs(X - X_ref[which]).max(axis=1) / np.maximum(1.0, np.abs(X_ref[which]).max(axis=1))
    _report("fullsize_partition_triangulation.json",
            dict(scene=s.name, n_points_checked=int(which.size), max_rel_err=float(err.max()),
                 n_failed_gpu=int(nf), n_failed_oracle_sample=int(nf_ref)))
    assert nf_ref == 0 and err.max() <= 1e-9
