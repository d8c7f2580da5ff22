"""FP64 CPU reference of the factorised sparse approximate inverse (FSAI)
preconditioner on the pattern of the reduced camera system (test
infrastructure only; shares no code with the HIP kernels).

The preconditioner is M^-1 = G^T G with G block-lower-triangular (9x9
blocks).  Block row i of G may be non-zero in the columns J_i: camera i
itself and the cameras s < i that share points with it (the lower half of
the RCS pattern, Eq. (4) and the BSMC pattern of Sec. 4).  When a row has
more such neighbours than a cap, the ones with the most common points are
kept (ties: lower index first).

Definition (Kolotilina and Yeremin's factorised sparse approximate inverse):
block row G_i is zero outside J_i and satisfies

    (G_i S)_j = 0  for j in J_i, j != i,      (G S G^T)_ii = I.

With the normalisation "G_ii lower triangular with positive diagonal" the
rows are unique.  Computed here straight from the definition: with
E_i the block column selecting camera i inside J_i,

    Y = S[J_i, J_i]^-1 E_i,   D = Y_i (the block of Y at i),
    C = chol(D^-1),            G_i = C^T Y^T.

The same G minimises the Kaporin functional
    f(G) = (tr(G S G^T) - 2 log det G) / (9 n)
over all block-lower-triangular G with that pattern and lower-triangular
diagonal blocks; `kaporin` evaluates it.

Storage convention (shared with the library's getter): G is returned in the
slots of the upper RCS blocks; the slot of upper block (s, c), s < c, holds
G_cs (block row c, block column s), the slot of a diagonal block holds G_ss.
Blocks of neighbours dropped by the cap are zero.
"""
from __future__ import annotations

import numpy as np


def shared_points(n_rows, cam_row, obs_cam, obs_pt):
    """Number of common points of every camera pair (r, s), r < s, as a dict,
    counted point by point from the observations."""
    cam_row = np.asarray(cam_row)
    obs_cam = np.asarray(obs_cam)
    obs_pt = np.asarray(obs_pt)
    order = np.lexsort((obs_cam, obs_pt))
    pts = obs_pt[order]
    rows = cam_row[obs_cam[order]]
    bounds = np.flatnonzero(np.diff(pts)) + 1
    cnt = {}
    for grp in np.split(rows, bounds):
        g = sorted(int(r) for r in grp if r >= 0)
        for a in range(len(g)):
            for b in range(a + 1, len(g)):
                key = (g[a], g[b])
                cnt[key] = cnt.get(key, 0) + 1
    return cnt


def lower_sets(rp, ci, strength, cap):
    """J_i (ascending, ending with i) of every row; `strength[(s, i)]` is the
    number of common points of cameras s < i; at most `cap` lower neighbours."""
    n = len(rp) - 1
    low = [[] for _ in range(n)]
    for r in range(n):
        for k in range(rp[r] + 1, rp[r + 1]):
            c = int(ci[k])
            low[c].append(r)
    out = []
    for i in range(n):
        cand = sorted(low[i], key=lambda s: (-strength[(s, i)], s))[:cap]
        out.append(sorted(cand) + [i])
    return out


def dense_rcs(blk, rp, ci):
    """Full symmetric S from upper blocks."""
    n = len(rp) - 1
    S = np.zeros((9 * n, 9 * n))
    for r in range(n):
        for k in range(rp[r], rp[r + 1]):
            c = int(ci[k])
            S[9 * r:9 * r + 9, 9 * c:9 * c + 9] = blk[k]
            S[9 * c:9 * c + 9, 9 * r:9 * r + 9] = blk[k].T
    return S


def fsai_rows(S, J):
    """Block rows G_i (each 9 x 9|J_i|) of the FSAI factor of dense S."""
    rows = []
    for i, Ji in enumerate(J):
        idx = np.concatenate([np.arange(9 * j, 9 * j + 9) for j in Ji])
        A = S[np.ix_(idx, idx)]
        E = np.zeros((len(idx), 9))
        pos = Ji.index(i)
        E[9 * pos:9 * pos + 9] = np.eye(9)
        Y = np.linalg.solve(A, E)
        D = Y[9 * pos:9 * pos + 9]
        D = 0.5 * (D + D.T)
        C = np.linalg.cholesky(np.linalg.inv(D))
        rows.append(C.T @ Y.T)
    return rows


def dense_factor(rows, J, n):
    G = np.zeros((9 * n, 9 * n))
    for i, (Gi, Ji) in enumerate(zip(rows, J)):
        for a, j in enumerate(Ji):
            G[9 * i:9 * i + 9, 9 * j:9 * j + 9] = Gi[:, 9 * a:9 * a + 9]
    return G


def slots_from_dense(G, rp, ci):
    """G in the upper-slot layout described in the module docstring."""
    n = len(rp) - 1
    out = np.zeros((int(rp[-1]), 9, 9))
    for r in range(n):
        for k in range(rp[r], rp[r + 1]):
            c = int(ci[k])
            out[k] = G[9 * c:9 * c + 9, 9 * r:9 * r + 9]
    return out


def dense_from_slots(Gs, rp, ci):
    n = len(rp) - 1
    G = np.zeros((9 * n, 9 * n))
    for r in range(n):
        for k in range(rp[r], rp[r + 1]):
            c = int(ci[k])
            G[9 * c:9 * c + 9, 9 * r:9 * r + 9] = Gs[k]
    return G


def fsai(blk, rp, ci, strength, cap):
    """Returns (G dense, G in upper slots, J)."""
    S = dense_rcs(blk, rp, ci)
    J = lower_sets(rp, ci, strength, cap)
    G = dense_factor(fsai_rows(S, J), J, len(rp) - 1)
    return G, slots_from_dense(G, rp, ci), J


def kaporin(G, S):
    """(tr(G S G^T) - 2 log det G) / N for block-lower-triangular G."""
    N = S.shape[0]
    d = np.diag(G)
    return (np.trace(G @ S @ G.T) - 2.0 * np.sum(np.log(d))) / N


def pcg(S_apply, b, M_apply, tol=1e-6, max_iter=1000):
    """Preconditioned CG with the recurrence of Sec. 3.2 (zero start, stop
    when |r_k| / |r_0| <= tol).  Returns (x, iterations, relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    r0 = np.linalg.norm(r)
    if r0 == 0.0:
        return x, 0, 0.0
    z = M_apply(r)
    d = z.copy()
    rz = r @ z
    for k in range(max_iter):
        q = S_apply(d)
        alpha = rz / (d @ q)
        x += alpha * d
        r -= alpha * q
        rel = np.linalg.norm(r) / r0
        if rel <= tol:
            return x, k + 1, rel
        z = M_apply(r)
        rz_new = r @ z
        d = z + (rz_new / rz) * d
        rz = rz_new
    return x, max_iter, np.linalg.norm(r) / r0
