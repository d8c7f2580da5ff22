"""Shared intrinsics: FP64 CPU reference (TEST INFRASTRUCTURE ONLY: called by
the test-suite; the product library never loads it and shares no code with
it).

The paper counts c = 11 unknowns per camera, 6 exterior and 5 interior
(Sec. 4.1), and its datasets have fewer physical cameras than images
(Table 2, "Cam." column): images taken by one physical camera share its
interior parameters.  Unknowns here:
  image i:           exterior e_i = [w (3) axis-angle, t (3)];
  physical camera k: interior q_k = [f, cx, cy, k1, k2];
  point p:           X_p (3).
Projection of point X in image i taken by camera k = img_cam[i]:
  P = R(w) X + t,  (x, y) = (P_x, P_y) / P_z,  d = 1 + k1 r^2 + k2 r^4,
  pixel = (f d x + cx, f d y + cy),  residual e = pixel - observed.
Camera-side unknowns are ordered: the 6 exterior parameters of every free
image (in image order), then the 5 interior parameters of every physical
camera.  The reduced camera system is the Schur complement of the damped
normal matrix over these unknowns (Eq. (1), (3)-(4)), formed point by point
(Sec. 5): S = U* - sum_p W_p V*_p^-1 W_p^T, b = l_c - sum_p W_p V*_p^-1 l_p,
with U = H_cc (which now couples an image's exterior block with its
camera's interior block), Marquardt damping A_kk (1 + lambda) on every
diagonal entry of U and V.

Jacobians are by forward-mode dual numbers (numpy arrays of derivatives in
14 directions: 6 exterior, 5 interior, 3 point), vectorised over
observations.
"""
from __future__ import annotations

import numpy as np

NE, NQ, NP = 6, 5, 3
ND = NE + NQ + NP


class Dual:
    """Values [n] with derivatives [n][ND]."""

    __slots__ = ("v", "d")

    def __init__(self, v, d):
        self.v = v
        self.d = d

    @staticmethod
    def const(v):
        v = np.asarray(v, dtype=np.float64)
        return Dual(v, np.zeros(v.shape + (ND,)))

    @staticmethod
    def var(v, k):
        x = Dual.const(v)
        x.d[..., k] = 1.0
        return x

    def __add__(self, o):
        o = o if isinstance(o, Dual) else Dual.const(np.broadcast_to(o, self.v.shape))
        return Dual(self.v + o.v, self.d + o.d)

    __radd__ = __add__

    def __sub__(self, o):
        o = o if isinstance(o, Dual) else Dual.const(np.broadcast_to(o, self.v.shape))
        return Dual(self.v - o.v, self.d - o.d)

    def __rsub__(self, o):
        return Dual.const(np.broadcast_to(o, self.v.shape)) - self

    def __mul__(self, o):
        if not isinstance(o, Dual):
            return Dual(self.v * o, self.d * np.asarray(o)[..., None])
        return Dual(self.v * o.v, self.d * o.v[..., None] + o.d * self.v[..., None])

    __rmul__ = __mul__

    def __truediv__(self, o):
        if not isinstance(o, Dual):
            return Dual(self.v / o, self.d / np.asarray(o)[..., None])
        q = self.v / o.v
        return Dual(q, (self.d - o.d * q[..., None]) / o.v[..., None])


def dsin(a):
    return Dual(np.sin(a.v), a.d * np.cos(a.v)[..., None])


def dsqrt(a):
    r = np.sqrt(a.v)
    return Dual(r, a.d / (2.0 * r)[..., None])


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _rotate(w, X):
    """Rodrigues: R X = X + sin(th) (k x X) + (1 - cos th) k x (k x X), k = w / th,
    with 1 - cos th = 2 sin^2(th / 2); w here is far from 0 (nadir cameras
    rotate by about pi), which the callers check."""
    th = dsqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2])
    k = [w[0] / th, w[1] / th, w[2] / th]
    kx = _cross(k, X)
    kkx = _cross(k, kx)
    sn = dsin(th)
    sh = dsin(th * 0.5)
    omc = sh * sh * 2.0
    return [X[i] + sn * kx[i] + omc * kkx[i] for i in range(3)]


def project(ext, intr, img_cam, pts, obs_img, obs_pt, with_jac=True):
    """Predicted pixels (u, v) of every observation as Duals in the 14
    directions [exterior (6), interior (5), point (3)]."""
    e = ext[obs_img]
    q = intr[img_cam[obs_img]]
    X = pts[obs_pt]
    if np.any(np.linalg.norm(e[:, :3], axis=1) < 1e-6):
        raise ValueError("rotation angle too close to 0 for this reference")
    w = [Dual.var(e[:, j], j) for j in range(3)]
    t = [Dual.var(e[:, 3 + j], 3 + j) for j in range(3)]
    f, cx, cy, k1, k2 = (Dual.var(q[:, j], NE + j) for j in range(5))
    Xd = [Dual.var(X[:, j], NE + NQ + j) for j in range(3)]
    P = _rotate(w, Xd)
    P = [P[i] + t[i] for i in range(3)]
    x = P[0] / P[2]
    y = P[1] / P[2]
    r2 = x * x + y * y
    d = 1.0 + k1 * r2 + k2 * (r2 * r2)
    return f * d * x + cx, f * d * y + cy


def linearize(ext, intr, img_cam, pts, obs_img, obs_pt, uv):
    """F = 1/2 sum |e|^2, e [n][2], Je [n][2][6], Jq [n][2][5], Jp [n][2][3]."""
    pu, pv = project(ext, intr, img_cam, pts, obs_img, obs_pt)
    e = np.stack([pu.v - uv[0], pv.v - uv[1]], axis=1)
    J = np.stack([pu.d, pv.d], axis=1)   # [n][2][14]
    return 0.5 * float(np.sum(e * e)), e, J[:, :, :NE], J[:, :, NE:NE + NQ], J[:, :, NE + NQ:]


class SharedProblem:
    """Observations (obs_img, obs_pt, uv) of n_img images taken by n_phys
    physical cameras (img_cam[i]); img_fixed marks images whose exterior is
    held fixed (their observations still count for the intrinsics and the
    points)."""

    def __init__(self, n_img, n_phys, img_cam, n_pts, obs_img, obs_pt, uv, img_fixed=None):
        self.n_img, self.n_phys, self.n_pts = n_img, n_phys, n_pts
        self.img_cam = np.asarray(img_cam, np.int64)
        self.obs_img = np.asarray(obs_img, np.int64)
        self.obs_pt = np.asarray(obs_pt, np.int64)
        self.uv = np.asarray(uv, np.float64)
        fixed = np.zeros(n_img, bool) if img_fixed is None else np.asarray(img_fixed, bool)
        self.img_row = np.full(n_img, -1, np.int64)
        self.img_row[~fixed] = np.arange(int((~fixed).sum()))
        self.n_free = int((~fixed).sum())
        self.m = NE * self.n_free + NQ * n_phys      # camera-side unknowns
        self.tracks = [np.nonzero(self.obs_pt == p)[0] for p in range(n_pts)]

    def ext_index(self, i):
        r = self.img_row[i]
        return None if r < 0 else np.arange(NE * r, NE * r + NE)

    def intr_index(self, k):
        return np.arange(NE * self.n_free + NQ * k, NE * self.n_free + NQ * k + NQ)

    def rcs(self, ext, intr, pts, lam):
        """Dense S [m][m] and b [m] of the damped system reduced over the
        points, formed point by point (Sec. 5), and F."""
        F, e, Je, Jq, Jp = linearize(ext, intr, self.img_cam, pts, self.obs_img, self.obs_pt, self.uv)
        m = self.m
        U = np.zeros((m, m))
        lc = np.zeros(m)
        S_minus = np.zeros((m, m))
        b_minus = np.zeros(m)
        for a in range(len(self.obs_img)):
            idx, Jc = self._cam_cols(a, Je, Jq)
            U[np.ix_(idx, idx)] += Jc.T @ Jc
            lc[idx] -= Jc.T @ e[a]
        for p in range(self.n_pts):
            tr = self.tracks[p]
            V = sum(Jp[a].T @ Jp[a] for a in tr)
            lp = -sum(Jp[a].T @ e[a] for a in tr)
            Vs = V + lam * np.diag(np.diag(V))
            Vi = np.linalg.inv(Vs)
            W = np.zeros((m, 3))
            for a in tr:
                idx, Jc = self._cam_cols(a, Je, Jq)
                W[idx] += Jc.T @ Jp[a]
            S_minus += W @ Vi @ W.T
            b_minus += W @ Vi @ lp
        Us = U + lam * np.diag(np.diag(U))
        return Us - S_minus, lc - b_minus, F

    def _cam_cols(self, a, Je, Jq):
        i = self.obs_img[a]
        qi = self.intr_index(self.img_cam[i])
        ei = self.ext_index(i)
        if ei is None:
            return qi, Jq[a]
        return np.concatenate([ei, qi]), np.concatenate([Je[a], Jq[a]], axis=1)

    def nodes_of_unknowns(self):
        """Node of each camera-side unknown and its slot in the node's padded
        9-vector: nodes are the free images (slots 0..5), then the physical
        cameras (slots 0..4)."""
        node = np.empty(self.m, np.int64)
        slot = np.empty(self.m, np.int64)
        node[:NE * self.n_free] = np.repeat(np.arange(self.n_free), NE)
        slot[:NE * self.n_free] = np.tile(np.arange(NE), self.n_free)
        node[NE * self.n_free:] = self.n_free + np.repeat(np.arange(self.n_phys), NQ)
        slot[NE * self.n_free:] = np.tile(np.arange(NQ), self.n_phys)
        return node, slot

    def pattern(self):
        """Upper node-block pattern (diagonal first, then ascending columns):
        block (u, v), u < v, is present iff some point is observed through
        both nodes (an image node and its own camera's node always are)."""
        n_nodes = self.n_free + self.n_phys
        pairs = set((u, u) for u in range(n_nodes))
        for p in range(self.n_pts):
            nodes = set()
            for a in self.tracks[p]:
                i = self.obs_img[a]
                if self.img_row[i] >= 0:
                    nodes.add(int(self.img_row[i]))
                nodes.add(self.n_free + int(self.img_cam[i]))
            nodes = sorted(nodes)
            for x in range(len(nodes)):
                for y in range(x + 1, len(nodes)):
                    pairs.add((nodes[x], nodes[y]))
        rows = [[] for _ in range(n_nodes)]
        for u, v in pairs:
            rows[u].append(v)
        row_ptr = np.zeros(n_nodes + 1, np.int64)
        col = []
        for u in range(n_nodes):
            r = sorted(rows[u])
            col.extend(r)
            row_ptr[u + 1] = len(col)
        return row_ptr, np.array(col, np.int32)

    def padded_blocks(self, S, b):
        """The dense RCS as padded 9x9 node blocks on the pattern: real
        entries in the node's slots, identity on the padding diagonal, zero
        padding elsewhere; rhs [n_nodes][9] with zero padding."""
        rp, ci = self.pattern()
        node, slot = self.nodes_of_unknowns()
        n_nodes = len(rp) - 1
        full = np.zeros((n_nodes, 9, n_nodes, 9))
        full[node[:, None], slot[:, None], node[None, :], slot[None, :]] = S
        for u in range(n_nodes):
            nreal = NE if u < self.n_free else NQ
            for c in range(nreal, 9):
                full[u, c, u, c] = 1.0
        blk = np.empty((len(ci), 9, 9))
        for u in range(n_nodes):
            for k in range(rp[u], rp[u + 1]):
                blk[k] = full[u, :, ci[k], :]
        rhs = np.zeros((n_nodes, 9))
        rhs[node, slot] = b
        return rp, ci, blk, rhs

    def dense_step(self, ext, intr, pts, lam):
        """Solution of the damped normal equations (Eq. (1)) over all unknowns
        by a dense solve: (dx_ext [n_img][6], dx_intr [n_phys][5],
        dx_pts [n_pts][3]), F, and the predicted decrease dx^T l - 1/2 |J dx|^2."""
        F, e, Je, Jq, Jp = linearize(ext, intr, self.img_cam, pts, self.obs_img, self.obs_pt, self.uv)
        m = self.m
        J = np.zeros((2 * len(self.obs_img), m + 3 * self.n_pts))
        for k in range(len(self.obs_img)):
            idx, Jc = self._cam_cols(k, Je, Jq)
            J[2 * k:2 * k + 2, idx] = Jc
            p = self.obs_pt[k]
            J[2 * k:2 * k + 2, m + 3 * p:m + 3 * p + 3] = Jp[k]
        H = J.T @ J
        g = -J.T @ e.ravel()
        A = H + lam * np.diag(np.diag(H))
        dx = np.linalg.solve(A, g)
        pred = float(dx @ g - 0.5 * np.sum((J @ dx) ** 2))
        dext = np.zeros((self.n_img, NE))
        for i in range(self.n_img):
            ei = self.ext_index(i)
            if ei is not None:
                dext[i] = dx[ei]
        dintr = np.stack([dx[self.intr_index(k)] for k in range(self.n_phys)])
        return dext, dintr, dx[m:].reshape(-1, 3), F, pred

    def cost(self, ext, intr, pts):
        return linearize(ext, intr, self.img_cam, pts, self.obs_img, self.obs_pt, self.uv)[0]


def lm_run(problem, ext, intr, pts, iterations, lam0=1e-4):
    """Fixed budget of LM iterations with exact steps (dense solves) and the
    damping schedule of the 9-parameter oracle: accept iff the predicted
    decrease is positive and F' < F; on accept lambda *= max(1/3,
    1 - (2 rho - 1)^3), nu = 2; on reject lambda *= nu, nu *= 2."""
    ext, intr, pts = ext.copy(), intr.copy(), pts.copy()
    lam, nu = lam0, 2.0
    hist = []
    for _ in range(iterations):
        dext, dintr, dpts, F, pred = problem.dense_step(ext, intr, pts, lam)
        Fn = problem.cost(ext + dext, intr + dintr, pts + dpts)
        rho = (F - Fn) / pred
        ok = pred > 0 and Fn < F
        if ok:
            ext, intr, pts = ext + dext, intr + dintr, pts + dpts
            lam *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            nu = 2.0
        else:
            lam *= nu
            nu *= 2.0
        hist.append(dict(cost=F, cost_new=Fn, accepted=int(ok), rho=rho, lambda_after=lam))
    return ext, intr, pts, hist
