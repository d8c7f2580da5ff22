"""Python binding of libba.so (argument marshalling only).

Every function mirrors the C entry point of the same name in include/ba.h.
Device arrays are torch tensors on the GPU (float64 / int32 / uint8, C
contiguous); work is ordered on torch's current HIP stream unless a stream
is given.  The library is required: importing this module on a machine
without the built library raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libba.so")

(BA_OK, BA_ERR_INVALID_ARG, BA_ERR_STATE, BA_ERR_NOT_SPD, BA_ERR_NOT_CONVERGED, BA_ERR_OUT_OF_MEMORY, BA_ERR_DEVICE,
 BA_ERR_RANGE) = range(8)
BA_FP64, BA_MIXED = 0, 1
BA_PRECOND_BLOCK_JACOBI, BA_PRECOND_LEARNED, BA_PRECOND_FSAI, BA_PRECOND_LEARNED_FSAI = 0, 1, 2, 3
BA_PRODUCT_AUTO, BA_PRODUCT_FULL, BA_PRODUCT_UPPER, BA_PRODUCT_CSR = 0, 1, 2, 3


class ProblemDesc(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("n_pts", C.c_int32), ("n_obs", C.c_int64),
                ("obs_cam", C.c_void_p), ("obs_pt", C.c_void_p), ("obs_uv", C.c_void_p),
                ("cam_fixed", C.c_void_p), ("precision", C.c_int32), ("reserved", C.c_int32),
                ("stream", C.c_void_p), ("workspace_cap", C.c_size_t)]


class SharedDesc(C.Structure):
    _fields_ = [("n_imgs", C.c_int32), ("n_phys", C.c_int32), ("n_pts", C.c_int32), ("reserved", C.c_int32),
                ("n_obs", C.c_int64), ("obs_img", C.c_void_p), ("obs_pt", C.c_void_p), ("obs_uv", C.c_void_p),
                ("img_cam", C.c_void_p), ("img_fixed", C.c_void_p), ("stream", C.c_void_p),
                ("workspace_cap", C.c_size_t)]


class PcgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("precond", C.c_int32), ("x0", C.c_void_p),
                ("deflate", C.c_int32), ("solver_fp32", C.c_int32), ("product", C.c_int32),
                ("reserved", C.c_int32)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("relres", C.c_double), ("ms", C.c_double),
                ("precond_fallback", C.c_int32), ("reserved", C.c_int32)]


class LMState(C.Structure):
    _fields_ = [("lam", C.c_double), ("nu", C.c_double), ("iter", C.c_int32), ("flags", C.c_int32)]


class LMOpts(C.Structure):
    _fields_ = [("pcg_tol", C.c_double), ("pcg_max_iter", C.c_int32), ("precond", C.c_int32),
                ("deflate", C.c_int32), ("solver_fp32", C.c_int32), ("product", C.c_int32),
                ("retriangulate", C.c_int32)]


class LMInfo(C.Structure):
    _fields_ = [("cost", C.c_double), ("cost_new", C.c_double), ("rho", C.c_double),
                ("model_decrease", C.c_double), ("pcg_relres", C.c_double),
                ("pcg_iters", C.c_int32), ("pcg_status", C.c_int32), ("accepted", C.c_int32),
                ("stop", C.c_int32), ("ms_linearize", C.c_double), ("ms_form_rcs", C.c_double),
                ("ms_pcg", C.c_double), ("ms_back_substitute", C.c_double),
                ("ms_evaluate", C.c_double), ("ms_total", C.c_double), ("ms_precond", C.c_double),
                ("precond_fallback", C.c_int32), ("tri_failed", C.c_int32)]


class Sizes(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("n_pts", C.c_int32), ("n_rows", C.c_int32), ("precision", C.c_int32),
                ("n_obs", C.c_int64), ("n_blk", C.c_int64), ("n_pairs", C.c_int64), ("device_bytes", C.c_int64)]


class StoreSizes(C.Structure):
    _fields_ = [("bsmc_bytes", C.c_int64), ("full_bytes", C.c_int64), ("csr_nnz", C.c_int64),
                ("csr_bytes", C.c_int64)]


# exported symbol -> (restype, argtypes)
_vp, _dp = C.c_void_p, C.POINTER(C.c_double)
SIGNATURES = {
    "ba_create": (C.c_int, [C.POINTER(ProblemDesc), C.POINTER(C.c_void_p)]),
    "ba_destroy": (None, [_vp]),
    "ba_create_shared": (C.c_int, [C.POINTER(SharedDesc), C.POINTER(C.c_void_p)]),
    "ba_linearize": (C.c_int, [_vp, _vp, _vp, _dp]),
    "ba_form_rcs": (C.c_int, [_vp, C.c_double]),
    "ba_pcg_solve": (C.c_int, [_vp, C.POINTER(PcgOpts), _vp, C.POINTER(PcgInfo)]),
    "ba_rcs_product": (C.c_int, [_vp, _vp, _vp, C.c_int32, C.c_int32]),
    "ba_back_substitute": (C.c_int, [_vp, _vp, _vp]),
    "ba_lm_step": (C.c_int, [_vp, _vp, _vp, C.POINTER(LMState), C.POINTER(LMOpts), C.POINTER(LMInfo)]),
    "ba_project": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int64, _vp, _vp, _vp]),
    "ba_triangulate": (C.c_int, [_vp, _vp, _vp, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]),
    "ba_cost_noalloc": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int64, _vp, _vp]),
    "ba_get_sizes": (C.c_int, [_vp, C.POINTER(Sizes)]),
    "ba_get_pattern": (C.c_int, [_vp, _vp, _vp]),
    "ba_get_rcs": (C.c_int, [_vp, _vp, _vp]),
    "ba_get_jacobians": (C.c_int, [_vp, _vp, _vp]),
    "ba_get_csr": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_int64)]),
    "ba_get_store_sizes": (C.c_int, [_vp, C.POINTER(StoreSizes)]),
    "ba_get_fsai": (C.c_int, [_vp, _vp]),
    "ba_get_gauge": (C.c_int, [_vp, _vp]),
    "ba_get_stage_ms": (C.c_int, [_vp, _dp]),
    "ba_status_str": (C.c_char_p, [C.c_int]),
    "ba_last_error": (C.c_char_p, [_vp]),
    "ba_gnn_param_count": (C.c_int64, []),
    "ba_gnn_create": (C.c_int, [_vp, _vp, C.POINTER(C.c_void_p)]),
    "ba_gnn_destroy": (None, [_vp]),
    "ba_gnn_set_params": (C.c_int, [_vp, _vp]),
    "ba_gnn_get_params": (C.c_int, [_vp, _vp]),
    "ba_gnn_graph_from_ctx": (C.c_int, [_vp, C.POINTER(C.c_void_p)]),
    "ba_gnn_graph_from_host": (C.c_int, [C.c_int32, _vp, _vp, _vp, _vp, C.POINTER(C.c_void_p)]),
    "ba_gnn_graph_destroy": (None, [_vp]),
    "ba_gnn_loss_grad": (C.c_int, [_vp, _vp, C.c_int32, _vp, C.c_uint64, _dp, _vp]),
    "ba_gnn_train_step": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, C.c_uint64, C.c_float, _dp]),
    "ba_gnn_preconditioner": (C.c_int, [_vp, _vp, _vp]),
    "ba_gnn_fsai_loss_grad": (C.c_int, [_vp, _vp, _dp, _vp]),
    "ba_gnn_fsai_train_step": (C.c_int, [_vp, _vp, C.c_int32, C.c_float, _dp]),
    "ba_gnn_fsai_factor": (C.c_int, [_vp, _vp, _vp]),
    "ba_set_preconditioner_net": (C.c_int, [_vp, _vp]),
    "ba_gemm_bf16": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp]),
    "ba_gnn_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class BAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib().ba_status_str(status).decode()}: {msg}")
        self.status = status


def _check(status, ctx=None, allow=()):
    if status != BA_OK and status not in allow:
        raise BAError(status, lib().ba_last_error(ctx).decode())
    return status


def _ptr(t):
    if t is None:
        return None
    assert t.is_contiguous(), "tensor must be contiguous"
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
def ba_create(n_cams, n_pts, obs_cam, obs_pt, obs_uv, cam_fixed=None, precision=BA_FP64,
              stream=None, workspace_cap=0):
    """obs_cam/obs_pt: int32 [n_obs]; obs_uv: float64 [2][n_obs]; cam_fixed: uint8 [n_cams] or None."""
    import torch
    assert obs_cam.dtype == torch.int32 and obs_pt.dtype == torch.int32 and obs_uv.dtype == torch.float64
    d = ProblemDesc(n_cams=n_cams, n_pts=n_pts, n_obs=obs_cam.numel(), obs_cam=_ptr(obs_cam),
                    obs_pt=_ptr(obs_pt), obs_uv=_ptr(obs_uv), cam_fixed=_ptr(cam_fixed),
                    precision=precision, reserved=0, stream=_stream(stream), workspace_cap=workspace_cap)
    h = C.c_void_p()
    _check(lib().ba_create(C.byref(d), C.byref(h)))
    return h


def ba_create_shared(n_imgs, n_phys, n_pts, obs_img, obs_pt, obs_uv, img_cam, img_fixed=None, stream=None,
                     workspace_cap=0):
    """Shared-intrinsics context: obs_img/obs_pt int32 [n_obs], obs_uv float64
    [2][n_obs], img_cam int32 [n_imgs], img_fixed uint8 [n_imgs] or None."""
    import torch
    assert obs_img.dtype == torch.int32 and obs_pt.dtype == torch.int32 and img_cam.dtype == torch.int32
    d = SharedDesc(n_imgs=n_imgs, n_phys=n_phys, n_pts=n_pts, reserved=0, n_obs=obs_img.numel(),
                   obs_img=_ptr(obs_img), obs_pt=_ptr(obs_pt), obs_uv=_ptr(obs_uv), img_cam=_ptr(img_cam),
                   img_fixed=_ptr(img_fixed), stream=_stream(stream), workspace_cap=workspace_cap)
    h = C.c_void_p()
    _check(lib().ba_create_shared(C.byref(d), C.byref(h)))
    return h


def ba_destroy(ctx):
    if ctx:
        lib().ba_destroy(ctx)


def ba_linearize(ctx, cams, pts, want_cost=True):
    cost = C.c_double(0.0)
    _check(lib().ba_linearize(ctx, _ptr(cams), _ptr(pts), C.byref(cost) if want_cost else None), ctx)
    return cost.value if want_cost else None


def ba_form_rcs(ctx, lam):
    _check(lib().ba_form_rcs(ctx, float(lam)), ctx)


def ba_pcg_solve(ctx, dxc, tol=1e-6, max_iter=1000, precond=BA_PRECOND_BLOCK_JACOBI, x0=None, deflate=False,
                 solver_fp32=False, product=BA_PRODUCT_AUTO):
    o = PcgOpts(tol=tol, max_iter=max_iter, precond=precond, x0=_ptr(x0), deflate=int(bool(deflate)),
                solver_fp32=int(bool(solver_fp32)), product=int(product))
    info = PcgInfo()
    st = _check(lib().ba_pcg_solve(ctx, C.byref(o), _ptr(dxc), C.byref(info)), ctx,
                allow=(BA_ERR_NOT_CONVERGED,))
    return dict(iters=info.iters, status=info.status, relres=info.relres, ms=info.ms,
                precond_fallback=info.precond_fallback, returned=st)


def ba_rcs_product(ctx, x, y, product=BA_PRODUCT_AUTO, solver_fp32=False):
    """y = S x (device [n_rows][9] tensors) as one PCG product would form it."""
    _check(lib().ba_rcs_product(ctx, _ptr(x), _ptr(y), int(product), int(bool(solver_fp32))), ctx)


def ba_back_substitute(ctx, dxc, dxp):
    _check(lib().ba_back_substitute(ctx, _ptr(dxc), _ptr(dxp)), ctx)


def ba_lm_step(ctx, cams, pts, state: LMState, pcg_tol=1e-6, pcg_max_iter=1000,
               precond=BA_PRECOND_BLOCK_JACOBI, deflate=False, solver_fp32=False, product=BA_PRODUCT_AUTO,
               retriangulate=0):
    o = LMOpts(pcg_tol=pcg_tol, pcg_max_iter=pcg_max_iter, precond=precond, deflate=int(bool(deflate)),
               solver_fp32=int(bool(solver_fp32)), product=int(product), retriangulate=int(retriangulate))
    info = LMInfo()
    _check(lib().ba_lm_step(ctx, _ptr(cams), _ptr(pts), C.byref(state), C.byref(o), C.byref(info)), ctx)
    return {k: getattr(info, k) for k, _ in LMInfo._fields_}


def ba_triangulate(ctx, cams, pts, linear_init=True, n_gn=5):
    """Re-triangulates every point in place (pts: device [n_pts][3]) with the
    cameras fixed; returns the number of points that failed."""
    nf = C.c_int64(0)
    _check(lib().ba_triangulate(ctx, _ptr(cams), _ptr(pts), int(bool(linear_init)), int(n_gn), C.byref(nf)), ctx)
    return nf.value


def ba_cost_noalloc(cams, pts, obs_cam, obs_pt, uv, cost, n_obs=None, stream=None):
    """F = 1/2 sum |e|^2 into the device scalar `cost` (float64 tensor of one
    element) without allocating; returns the status (BA_OK or an error)."""
    n = obs_cam.numel() if n_obs is None else n_obs
    return lib().ba_cost_noalloc(_ptr(cams), _ptr(pts), _ptr(obs_cam), _ptr(obs_pt), _ptr(uv), n, _ptr(cost),
                                 _stream(stream))


def ba_project(cams, pts, obs_cam, obs_pt, noise=None, out=None, stream=None):
    import torch
    n = obs_cam.numel()
    uv = out if out is not None else torch.empty((2, n), dtype=torch.float64, device=cams.device)
    _check(lib().ba_project(_ptr(cams), _ptr(pts), _ptr(obs_cam), _ptr(obs_pt), n, _ptr(noise),
                            _ptr(uv), _stream(stream)))
    return uv


def ba_get_sizes(ctx):
    s = Sizes()
    _check(lib().ba_get_sizes(ctx, C.byref(s)), ctx)
    return {k: getattr(s, k) for k, _ in Sizes._fields_}


def ba_get_pattern(ctx):
    s = ba_get_sizes(ctx)
    rp = np.empty(s["n_rows"] + 1, np.int64)
    ci = np.empty(max(s["n_blk"], 1), np.int32)
    _check(lib().ba_get_pattern(ctx, _np_ptr(rp), _np_ptr(ci)), ctx)
    return rp, ci[: s["n_blk"]]


def ba_get_rcs(ctx):
    s = ba_get_sizes(ctx)
    blk = np.empty((max(s["n_blk"], 1), 9, 9))
    rhs = np.empty((max(s["n_rows"], 1), 9))
    _check(lib().ba_get_rcs(ctx, _np_ptr(blk), _np_ptr(rhs)), ctx)
    return blk[: s["n_blk"]], rhs[: s["n_rows"]]


def ba_get_jacobians(ctx):
    """Returns (J [n_obs][24], e [n_obs][2]) in the caller's observation order."""
    s = ba_get_sizes(ctx)
    J = np.empty((s["n_obs"], 24))
    e = np.empty((s["n_obs"], 2))
    _check(lib().ba_get_jacobians(ctx, _np_ptr(J), _np_ptr(e)), ctx)
    return J, e


def ba_get_store_sizes(ctx):
    s = StoreSizes()
    _check(lib().ba_get_store_sizes(ctx, C.byref(s)), ctx)
    return {k: getattr(s, k) for k, _ in StoreSizes._fields_}


def ba_get_csr(ctx):
    """CSR copy of the last formed RCS: (row_ptr [9 n_rows + 1], col, val)."""
    s = ba_get_sizes(ctx)
    nnz = C.c_int64(0)
    _check(lib().ba_get_csr(ctx, None, None, None, C.byref(nnz)), ctx)
    rp = np.empty(9 * s["n_rows"] + 1, np.int32)
    col = np.empty(max(nnz.value, 1), np.int32)
    val = np.empty(max(nnz.value, 1))
    _check(lib().ba_get_csr(ctx, _np_ptr(rp), _np_ptr(col), _np_ptr(val), None), ctx)
    return rp, col[: nnz.value], val[: nnz.value]


def ba_get_gauge(ctx):
    """Gauge vectors of the last linearization, FP64 [n_rows][7][9]."""
    s = ba_get_sizes(ctx)
    W = np.empty((max(s["n_rows"], 1), 7, 9))
    _check(lib().ba_get_gauge(ctx, _np_ptr(W)), ctx)
    return W[: s["n_rows"]]


def ba_get_fsai(ctx):
    """FSAI factor of the current RCS, FP32 [n_blk][9][9] in the RCS block slots."""
    s = ba_get_sizes(ctx)
    G = np.empty((max(s["n_blk"], 1), 9, 9), np.float32)
    _check(lib().ba_get_fsai(ctx, _np_ptr(G)), ctx)
    return G[: s["n_blk"]]


def ba_get_stage_ms(ctx):
    ms = (C.c_double * 4)()
    _check(lib().ba_get_stage_ms(ctx, ms), ctx)
    return list(ms)


def ba_status_str(status):
    return lib().ba_status_str(status).decode()


def ba_last_error(ctx=None):
    return lib().ba_last_error(ctx).decode()


def new_lm_state(lam=1e-4):
    return LMState(lam=lam, nu=2.0, iter=0, flags=0)


# ---------------------------------------------------------------------------
# learned preconditioner
# ---------------------------------------------------------------------------
def _gnn_check(status):
    if status != BA_OK:
        raise BAError(status, lib().ba_gnn_last_error().decode())
    return status


def ba_gnn_param_count():
    return int(lib().ba_gnn_param_count())


def ba_gnn_create(params, stream=None):
    """params: float32 host array of ba_gnn_param_count() values."""
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == ba_gnn_param_count()
    h = C.c_void_p()
    st = None if stream is None else C.c_void_p(stream.cuda_stream)
    _gnn_check(lib().ba_gnn_create(_np_ptr(p), st, C.byref(h)))
    return h


def ba_gnn_destroy(net):
    if net:
        lib().ba_gnn_destroy(net)


def ba_gnn_set_params(net, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _gnn_check(lib().ba_gnn_set_params(net, _np_ptr(p)))


def ba_gnn_get_params(net):
    out = np.empty(ba_gnn_param_count(), np.float32)
    _gnn_check(lib().ba_gnn_get_params(net, _np_ptr(out)))
    return out


def ba_gnn_graph_from_ctx(ctx):
    h = C.c_void_p()
    _check(lib().ba_gnn_graph_from_ctx(ctx, C.byref(h)), ctx)
    return h


def ba_gnn_graph_from_host(row_ptr, col_idx, blk, blk_pairs=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    b = np.ascontiguousarray(blk, dtype=np.float64)
    bp = None if blk_pairs is None else np.ascontiguousarray(blk_pairs, dtype=np.int32)
    h = C.c_void_p()
    _gnn_check(lib().ba_gnn_graph_from_host(len(rp) - 1, _np_ptr(rp), _np_ptr(ci), _np_ptr(b), _np_ptr(bp),
                                            C.byref(h)))
    return h


def ba_gnn_graph_destroy(g):
    if g:
        lib().ba_gnn_graph_destroy(g)


def ba_gnn_loss_grad(net, graph, n_probes=4, probes=None, seed=0, want_grad=True):
    loss = C.c_double(0.0)
    pr = None if probes is None else np.ascontiguousarray(probes, dtype=np.float32)
    grad = np.empty(ba_gnn_param_count(), np.float32) if want_grad else None
    _gnn_check(lib().ba_gnn_loss_grad(net, graph, n_probes, _np_ptr(pr), seed, C.byref(loss), _np_ptr(grad)))
    return loss.value, grad


def ba_gnn_train_step(net, graphs, n_probes=4, seed=0, lr=1e-3):
    arr = (C.c_void_p * len(graphs))(*[g.value if isinstance(g, C.c_void_p) else g for g in graphs])
    loss = C.c_double(0.0)
    _gnn_check(lib().ba_gnn_train_step(net, arr, len(graphs), n_probes, seed, lr, C.byref(loss)))
    return loss.value


def ba_gnn_preconditioner(net, graph, n_rows):
    P = np.empty((n_rows, 9, 9))
    _gnn_check(lib().ba_gnn_preconditioner(net, graph, _np_ptr(P)))
    return P


def ba_gnn_fsai_loss_grad(net, graph, want_grad=True):
    loss = C.c_double(0.0)
    grad = np.empty(ba_gnn_param_count(), np.float32) if want_grad else None
    _gnn_check(lib().ba_gnn_fsai_loss_grad(net, graph, C.byref(loss), _np_ptr(grad)))
    return loss.value, grad


def ba_gnn_fsai_train_step(net, graphs, lr=1e-3):
    arr = (C.c_void_p * len(graphs))(*[g.value if isinstance(g, C.c_void_p) else g for g in graphs])
    loss = C.c_double(0.0)
    _gnn_check(lib().ba_gnn_fsai_train_step(net, arr, len(graphs), lr, C.byref(loss)))
    return loss.value


def ba_gnn_fsai_factor(net, graph, n_blk):
    """The head's factor G (FP32 [n_blk][9][9] in the RCS block slots)."""
    G = np.zeros((max(n_blk, 1), 9, 9), np.float32)
    _gnn_check(lib().ba_gnn_fsai_factor(net, graph, _np_ptr(G)))
    return G[:n_blk]


def ba_set_preconditioner_net(ctx, net):
    _check(lib().ba_set_preconditioner_net(ctx, net), ctx)


def ba_gemm_bf16(A_bits, B_bits):
    """A_bits [M][K], B_bits [K][N]: uint16 bf16 bit patterns; returns C float32."""
    A = np.ascontiguousarray(A_bits, dtype=np.uint16)
    B = np.ascontiguousarray(B_bits, dtype=np.uint16)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    Cm = np.empty((M, N), np.float32)
    _gnn_check(lib().ba_gemm_bf16(M, N, K, _np_ptr(A), _np_ptr(B), _np_ptr(Cm)))
    return Cm
