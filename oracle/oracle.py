"""ctypes wrapper around the C oracle (liboracle.so).

Test infrastructure only.  Array conventions follow the C side:
  cams [n_cams][9], pts [n_pts][3], uv [2][n_obs], e [n_obs][2],
  Jc [n_obs][2][9], Jp [n_obs][2][3], RCS blocks [n_blk][9][9] (upper
  triangle, diagonal first in each row), rhs / dxc [n_rows][9].
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


class LMState(C.Structure):
    _fields_ = [("lam", C.c_double), ("nu", C.c_double), ("iter", C.c_int32), ("pad", C.c_int32)]


class LMInfo(C.Structure):
    _fields_ = [("cost", C.c_double), ("cost_new", C.c_double), ("rho", C.c_double),
                ("model_decrease", C.c_double), ("pcg_relres", C.c_double),
                ("accepted", C.c_int32), ("pcg_iters", C.c_int32),
                ("pcg_status", C.c_int32), ("stop", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        vp = C.c_void_p
        L.orc_project.argtypes = [C.c_int64, _f64p, _f64p, _i32p, _i32p, vp, _f64p]
        L.orc_linearize.argtypes = [C.c_int64, _f64p, _f64p, _i32p, _i32p, _f64p, vp, vp, vp]
        L.orc_linearize.restype = C.c_double
        L.orc_create.argtypes = [C.c_int32, C.c_int32, C.c_int64, _i32p, _i32p, _f64p, vp, C.c_int32]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_n_rows.argtypes = [vp]; L.orc_n_rows.restype = C.c_int32
        L.orc_n_blk.argtypes = [vp]; L.orc_n_blk.restype = C.c_int64
        L.orc_get_pattern.argtypes = [vp, _i64p, _i32p]
        L.orc_get_cam_row.argtypes = [vp, _i32p]
        L.orc_prob_linearize.argtypes = [vp, _f64p, _f64p]
        L.orc_prob_linearize.restype = C.c_double
        L.orc_get_linearization.argtypes = [vp, vp, vp, vp]
        L.orc_form_rcs.argtypes = [vp, C.c_double, C.c_int32]
        L.orc_form_rcs.restype = C.c_int
        L.orc_get_rcs.argtypes = [vp, vp, vp]
        L.orc_set_rcs.argtypes = [vp, vp, vp]
        L.orc_get_point_terms.argtypes = [vp, vp, vp]
        L.orc_pcg.argtypes = [vp, C.c_double, C.c_int32, vp, vp, _f64p,
                              C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.orc_pcg.restype = C.c_int
        L.orc_spmv.argtypes = [vp, _f64p, _f64p]
        L.orc_back_substitute.argtypes = [vp, _f64p, _f64p]
        L.orc_cost.argtypes = [vp, _f64p, _f64p]
        L.orc_cost.restype = C.c_double
        L.orc_model_terms.argtypes = [vp, _f64p, _f64p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_lm_step.argtypes = [vp, _f64p, _f64p, C.POINTER(LMState), C.POINTER(LMInfo),
                                  C.c_double, C.c_int32]
        L.orc_lm_step.restype = C.c_int
        L.orc_triangulate.argtypes = [vp, _f64p, _f64p, _f64p, vp, C.c_int64, C.c_int32, C.c_int32]
        L.orc_triangulate.restype = C.c_int64
        L.orc_bsmc_bytes.argtypes = [vp, C.c_int32]
        L.orc_bsmc_bytes.restype = C.c_int64
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def default_threads():
    """Host threads for the oracle: OMP_NUM_THREADS when set, else all cores."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return os.cpu_count() or 1


def project(cams, pts, obs_cam, obs_pt, noise=None):
    """Observed pixels [2][n_obs] = projection(params) (+ noise)."""
    obs_cam = _c(obs_cam, np.int32)
    n = obs_cam.size
    uv = np.empty((2, n))
    nz = None if noise is None else _c(noise, np.float64)
    lib().orc_project(n, _c(cams, np.float64), _c(pts, np.float64), obs_cam,
                      _c(obs_pt, np.int32), _ptr(nz), uv)
    return uv


def linearize(cams, pts, obs_cam, obs_pt, uv):
    """Returns (F, e [n][2], Jc [n][2][9], Jp [n][2][3])."""
    obs_cam = _c(obs_cam, np.int32)
    n = obs_cam.size
    e = np.empty((n, 2)); Jc = np.empty((n, 2, 9)); Jp = np.empty((n, 2, 3))
    F = lib().orc_linearize(n, _c(cams, np.float64), _c(pts, np.float64), obs_cam,
                            _c(obs_pt, np.int32), _c(uv, np.float64), _ptr(e), _ptr(Jc), _ptr(Jp))
    return F, e, Jc, Jp


def observations(scene, cams=None, pts=None):
    """uv of a scene: its true parameters projected, plus its pixel noise."""
    return project(scene.cams_true if cams is None else cams,
                   scene.pts_true if pts is None else pts,
                   scene.obs_cam, scene.obs_pt, scene.noise)


class Problem:
    """Oracle problem: pattern, linearization, RCS, PCG, back-substitution, LM."""

    def __init__(self, n_cams, n_pts, obs_cam, obs_pt, uv, cam_fixed=None, n_threads=None):
        self._keep = (_c(obs_cam, np.int32), _c(obs_pt, np.int32), _c(uv, np.float64),
                      None if cam_fixed is None else _c(cam_fixed, np.uint8))
        n_obs = self._keep[0].size
        nt = n_threads or default_threads()
        h = lib().orc_create(n_cams, n_pts, n_obs, self._keep[0], self._keep[1], self._keep[2],
                             _ptr(self._keep[3]), nt)
        if not h:
            raise ValueError("invalid bundle-adjustment problem")
        self.h = h
        self.n_cams, self.n_pts, self.n_obs = n_cams, n_pts, n_obs
        self.n_rows = lib().orc_n_rows(h)
        self.n_blk = lib().orc_n_blk(h)

    @classmethod
    def from_scene(cls, scene, uv=None, n_threads=None):
        uv = observations(scene) if uv is None else uv
        return cls(scene.n_cams, scene.n_pts, scene.obs_cam, scene.obs_pt, uv,
                   scene.cam_fixed if scene.cam_fixed.any() else None, n_threads)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def pattern(self):
        rp = np.empty(self.n_rows + 1, np.int64)
        ci = np.empty(max(self.n_blk, 1), np.int32)
        lib().orc_get_pattern(self.h, rp, ci)
        return rp, ci[: self.n_blk]

    def cam_row(self):
        out = np.empty(self.n_cams, np.int32)
        lib().orc_get_cam_row(self.h, out)
        return out

    def linearize(self, cams, pts):
        return lib().orc_prob_linearize(self.h, _c(cams, np.float64), _c(pts, np.float64))

    def linearization(self):
        e = np.empty((self.n_obs, 2)); Jc = np.empty((self.n_obs, 2, 9)); Jp = np.empty((self.n_obs, 2, 3))
        lib().orc_get_linearization(self.h, _ptr(e), _ptr(Jc), _ptr(Jp))
        return e, Jc, Jp

    def form_rcs(self, lam, n_groups=0):
        rc = lib().orc_form_rcs(self.h, float(lam), int(n_groups))
        if rc != 0:
            raise RuntimeError(f"oracle form_rcs failed ({rc})")

    def rcs(self):
        blk = np.empty((max(self.n_blk, 1), 9, 9)); rhs = np.empty((max(self.n_rows, 1), 9))
        lib().orc_get_rcs(self.h, _ptr(blk), _ptr(rhs))
        return blk[: self.n_blk], rhs[: self.n_rows]

    def set_rcs(self, blk, rhs):
        blk = _c(blk, np.float64); rhs = _c(rhs, np.float64)
        lib().orc_set_rcs(self.h, _ptr(blk), _ptr(rhs))

    def point_terms(self):
        Vinv = np.empty((self.n_pts, 3, 3)); lp = np.empty((self.n_pts, 3))
        lib().orc_get_point_terms(self.h, _ptr(Vinv), _ptr(lp))
        return Vinv, lp

    def pcg(self, tol=1e-6, max_iter=1000, x0=None, M=None):
        x = np.empty((self.n_rows, 9))
        it = C.c_int32(0); rr = C.c_double(0)
        x0c = None if x0 is None else _c(x0, np.float64)
        Mc = None if M is None else _c(M, np.float64)
        st = lib().orc_pcg(self.h, float(tol), int(max_iter), _ptr(x0c), _ptr(Mc), x,
                           C.byref(it), C.byref(rr))
        return x, dict(status=st, iters=it.value, relres=rr.value)

    def spmv(self, x):
        y = np.empty((self.n_rows, 9))
        lib().orc_spmv(self.h, _c(x, np.float64).reshape(-1, 9), y)
        return y

    def back_substitute(self, dxc):
        dxp = np.empty((self.n_pts, 3))
        lib().orc_back_substitute(self.h, _c(dxc, np.float64), dxp)
        return dxp

    def cost(self, cams, pts):
        return lib().orc_cost(self.h, _c(cams, np.float64), _c(pts, np.float64))

    def model_terms(self, dxc, dxp):
        a = C.c_double(0); b = C.c_double(0)
        lib().orc_model_terms(self.h, _c(dxc, np.float64), _c(dxp, np.float64), C.byref(a), C.byref(b))
        return a.value, b.value

    def lm_step(self, cams, pts, state: LMState, tol=1e-6, max_iter=1000):
        """One LM iteration; cams/pts (float64, C-contiguous) updated in place on accept."""
        info = LMInfo()
        lib().orc_lm_step(self.h, cams, pts, C.byref(state), C.byref(info), float(tol), int(max_iter))
        return {k: getattr(info, k) for k, _ in LMInfo._fields_}

    def triangulate(self, cams, pts_start, init=True, n_gn=5, which=None):
        """Points re-estimated with the cameras fixed (linear start when init,
        then n_gn Gauss-Newton steps); returns (pts [n_pts][3], n_failed).
        Points outside `which` (when given) keep their start values."""
        out = np.array(pts_start, dtype=np.float64, order="C")
        w = None if which is None else _c(which, np.int32)
        nf = lib().orc_triangulate(self.h, _c(cams, np.float64), _c(pts_start, np.float64), out, _ptr(w),
                                   0 if w is None else w.size, int(bool(init)), int(n_gn))
        return out, int(nf)

    def bsmc_bytes(self, c=9):
        return lib().orc_bsmc_bytes(self.h, c)


def lm_run(problem: Problem, cams, pts, iterations, lam0=1e-4, tol=1e-6, max_iter=1000):
    """Fixed budget of LM iterations from (cams, pts); returns (cams, pts, history)."""
    cams = np.array(cams, dtype=np.float64, order="C")
    pts = np.array(pts, dtype=np.float64, order="C")
    st = LMState(lam=lam0, nu=2.0, iter=0, pad=0)
    hist = []
    for _ in range(iterations):
        info = problem.lm_step(cams, pts, st, tol, max_iter)
        info["lambda_after"] = st.lam
        hist.append(info)
        if info["stop"]:
            break
    return cams, pts, hist
