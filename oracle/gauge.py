"""FP64 CPU reference of the gauge-deflated PCG (test infrastructure only;
shares no code with the HIP kernels).

Gauge.  Projection (Eq. (1)'s residuals) is unchanged when the whole scene
undergoes a similarity transform X -> (1 + s) Q X + u, with every camera
adjusted so that its camera-frame coordinates only scale: R' = R Q^T,
t' = (1 + s) t - R Q^T u.  The seven infinitesimal generators therefore give
exact null vectors of J (Eq. (1)), and their camera parts are null vectors
of the undamped reduced camera system (Eq. (4)).  Per camera, with the
9-vector [w, t, f, k1, k2]:
  translation u = e_k:  dt = -R e_k                      (k = 0, 1, 2)
  scale s:              dt = t
  rotation Q = exp(-eps [e_k]x): dw = d/deps w(R exp(-eps [e_k]x))
Here the rotation part is taken by central differences of this module's
own Rodrigues map (dw solves R(w) exp(-eps [e_k]x) = R(w + eps dw) to first
order), intrinsics do not move.  Fixed cameras have no RCS rows.

Deflated CG (Saad, Yeung, Erhel and Guyomarc'h's deflated conjugate
gradient, Nicolaides' deflation) with deflation space W (columns above),
E = W^T S W and preconditioner M^-1:
  x0 = x_s + W E^-1 W^T r_s, r0 = b - S x0 (W^T r0 = 0), z0 = M^-1 r0,
  p0 = z0 - W E^-1 (S W)^T z0; per step alpha = r^T z / p^T S p,
  x += alpha p, r -= alpha S p, stop at |r| / |b - S x_s| <= tol,
  z = M^-1 r, beta = r'^T z' / r^T z, p = z' + beta p - W E^-1 (S W)^T z'.
The iterate converges to S^-1 b like plain PCG; only the path differs.
"""
from __future__ import annotations

import numpy as np


def _skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def rodrigues(w):
    th = np.linalg.norm(w)
    K = _skew(w)
    if th < 1e-8:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / th ** 2 * (K @ K)


def _vee(M):
    return 0.5 * np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])


def gauge_vectors(cams, cam_row, n_rows, h=1e-6):
    """W [n_rows * 9][7]: columns rotation x, y, z, translation x, y, z, scale."""
    W = np.zeros((9 * n_rows, 7))
    for c, r in enumerate(cam_row):
        if r < 0:
            continue
        w = np.asarray(cams[c, :3], dtype=np.float64)
        t = np.asarray(cams[c, 3:6], dtype=np.float64)
        R = rodrigues(w)
        # right Jacobian J_r: R(w + d) = R(w) exp([J_r d]x) to first order
        Jr = np.stack([_vee(R.T @ (rodrigues(w + h * e) - rodrigues(w - h * e)) / (2 * h))
                       for e in np.eye(3)], axis=1)
        dw = -np.linalg.inv(Jr)
        W[9 * r:9 * r + 3, 0:3] = dw
        W[9 * r + 3:9 * r + 6, 3:6] = -R
        W[9 * r + 3:9 * r + 6, 6] = t
    return W


def deflated_pcg(S_apply, b, M_apply, W, tol=1e-6, max_iter=1000, x_start=None):
    """Returns (x, iterations, relative residual, max_k |W^T r_k| / |r_0|)."""
    SW = np.stack([S_apply(W[:, j]) for j in range(W.shape[1])], axis=1)
    E = W.T @ SW
    Ei = np.linalg.inv(E)
    x = np.zeros_like(b) if x_start is None else np.array(x_start, dtype=np.float64)
    rs = b - S_apply(x) if x_start is not None else b.copy()
    y = Ei @ (W.T @ rs)
    x = x + W @ y
    r = rs - SW @ y
    r0 = np.linalg.norm(rs)
    if r0 == 0.0:
        return x, 0, 0.0, 0.0
    worst = np.linalg.norm(W.T @ r) / r0
    z = M_apply(r)
    p = z - W @ (Ei @ (SW.T @ z))
    rz = r @ z
    for k in range(max_iter):
        q = S_apply(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        worst = max(worst, np.linalg.norm(W.T @ r) / r0)
        rel = np.linalg.norm(r) / r0
        if rel <= tol:
            return x, k + 1, rel, worst
        z = M_apply(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p - W @ (Ei @ (SW.T @ z))
        rz = rz_new
    return x, max_iter, np.linalg.norm(r) / r0, worst
