"""FP64 CPU reference of the learned block-Jacobi correction (test
infrastructure only; shares no code with the HIP kernels).

The network runs on the camera-pair graph of the reduced camera system
(Eq. (4); its non-zero blocks are the camera pairs with common points, Sec. 4)
and outputs, per camera i, a lower-triangular 9x9 factor Lt_i (diagonal
exp(.)); the preconditioner block is

    P_i = L_i^-T (Lt_i Lt_i^T) L_i^-1,     S_ii = L_i L_i^T,

which is SPD by construction and equals the block-Jacobi inverse S_ii^-1
when Lt_i = I (zero decoder).  Training minimises the Hutchinson estimate of
||B A - I||_F^2 / (9 n) in the block-Jacobi-normalised space
A = blockdiag(L)^-1 S blockdiag(L)^-T, B = blockdiag(Lt Lt^T):

    loss = sum_p sum_i |B_i y_i^p - z_i^p|^2 / (n_probes 9 n),  y^p = A z^p.

Features (both sides compute them from the RCS):
  node i (64, 45 used): the 36 strictly-upper entries of the Jacobi-scaled
      diagonal block D S_ii D (D = diag(S_ii)^-1/2), then the 9 values
      log S_ii[r][r] minus their mean over r.
  directed edge i->j (96, 81 used): A_ij row-major (A_ji = A_ij^T).
Network (hidden 64): h = relu(x Wn + bn); g = relu(e We + be); three layers
  m_ij = relu([h_i, h_j, g_ij] M_l + c_l), a_i = mean_j m_ij,
  h_i += relu([h_i, a_i] U_l + u_l); output o = h Wd + bd (48, 45 used):
  o[0..8] -> diagonal exp(o), o[9..44] -> strict lower triangle row-major.
"""
from __future__ import annotations

import numpy as np

H = 64
F_NODE, F_EDGE, F_OUT = 64, 96, 48
N_LAYERS = 3

# flat parameter layout: (name, shape) in order
PARAM_SHAPES = [("Wn", (F_NODE, H)), ("bn", (H,)), ("We", (F_EDGE, H)), ("be", (H,))]
for _l in range(N_LAYERS):
    PARAM_SHAPES += [(f"M{_l}", (3 * H, H)), (f"c{_l}", (H,)), (f"U{_l}", (2 * H, H)), (f"u{_l}", (H,))]
PARAM_SHAPES += [("Wd", (H, F_OUT)), ("bd", (F_OUT,))]
# factorised head: off-diagonal blocks of G from [h_i, h_j, g_ij] through one
# hidden ReLU layer (96 outputs, 81 used) plus a learned elementwise multiple
# of the normalised block
F_OFF = 96
HO = 128
PARAM_SHAPES += [("Wo1", (3 * H, HO)), ("bo1", (HO,)), ("Wo2", (HO, F_OFF)), ("bo2", (F_OFF,)),
                 ("ao", (F_OFF,))]
N_PARAMS = int(sum(np.prod(s) for _, s in PARAM_SHAPES))

# strict lower triangle positions (row-major) used by the decoder
TRIL = [(r, c) for r in range(9) for c in range(r)]
TRIU = [(r, c) for r in range(9) for c in range(r + 1, 9)]


def unflatten(w):
    out, o = {}, 0
    for name, shape in PARAM_SHAPES:
        n = int(np.prod(shape))
        out[name] = w[o:o + n].reshape(shape)
        o += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in PARAM_SHAPES])


def init_params(seed=0, zero_decoder=True, decoder_scale=0.05):
    """Random weights with std 1/sqrt(fan_in) (update layers halved), zero
    biases; zero decoder => P = block-Jacobi."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in PARAM_SHAPES:
        if len(shape) == 2:
            scale = 0.5 if name[0] == "U" else 1.0
            d[name] = rng.normal(0.0, scale / np.sqrt(shape[0]), size=shape)
        else:
            d[name] = np.zeros(shape)
    if zero_decoder:
        d["Wd"][:] = 0.0
        d["bd"][:] = 0.0
        d["Wo2"][:] = 0.0
    else:
        d["Wd"] *= decoder_scale
        d["Wo2"] *= decoder_scale
    return flatten(d)


def bf16_round(x):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# graph and features
# ---------------------------------------------------------------------------

def graph_from_pattern(row_ptr, col_idx):
    """Directed edges i->j for every stored off-diagonal block (both
    directions), grouped by source, ascending destination; returns
    (edge_ptr, src, dst, blk, transposed, twin)."""
    n = len(row_ptr) - 1
    edges = []
    for r in range(n):
        for k in range(row_ptr[r], row_ptr[r + 1]):
            s = int(col_idx[k])
            if s != r:
                edges.append((r, s, k, 0))
                edges.append((s, r, k, 1))
    edges.sort(key=lambda t: (t[0], t[1]))
    src = np.array([e[0] for e in edges], dtype=np.int64)
    dst = np.array([e[1] for e in edges], dtype=np.int64)
    blk = np.array([e[2] for e in edges], dtype=np.int64)
    tr = np.array([e[3] for e in edges], dtype=np.int64)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, src + 1, 1)
    ptr = np.cumsum(ptr)
    index = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(src, dst))}
    twin = np.array([index[(int(b), int(a))] for a, b in zip(src, dst)], dtype=np.int64)
    return dict(ptr=ptr, src=src, dst=dst, blk=blk, tr=tr, twin=twin, n=n)


def features(row_ptr, col_idx, blk):
    """Cholesky factors, normalised blocks and the network inputs."""
    n = len(row_ptr) - 1
    g = graph_from_pattern(row_ptr, col_idx)
    L = np.zeros((n, 9, 9))
    xn = np.zeros((n, F_NODE))
    for i in range(n):
        S = blk[row_ptr[i]]
        L[i] = np.linalg.cholesky(S)
        d = 1.0 / np.sqrt(np.diag(S))
        Sh = S * d[:, None] * d[None, :]
        xn[i, :36] = [Sh[r, c] for r, c in TRIU]
        ld = np.log(np.diag(S))
        xn[i, 36:45] = ld - ld.mean()
    E = len(g["src"])
    A = np.zeros((E, 9, 9))
    for e in range(E):
        i, j, k = g["src"][e], g["dst"][e], g["blk"][e]
        Sij = blk[k] if g["tr"][e] == 0 else blk[k].T      # block (i, j) of S
        A[e] = np.linalg.solve(L[i], np.linalg.solve(L[j], Sij.T).T)   # L_i^-1 S_ij L_j^-T
    xe = np.zeros((E, F_EDGE))
    xe[:, :81] = A.reshape(E, 81)
    return dict(graph=g, L=L, A=A, xn=xn, xe=xe)


def normalised_product(feat, z):
    """y = A z with A_ii = I and A_ij on the directed edges; z: [n, 9]."""
    g, A = feat["graph"], feat["A"]
    y = z.copy()
    for e in range(len(g["src"])):
        y[g["src"][e]] += A[e] @ z[g["dst"][e]]
    return y


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def _relu(x):
    return np.maximum(x, 0.0)


def _params(w, bf16):
    """Weight matrices in bfloat16 and biases in FP32 (as the GPU keeps
    them) when bf16, otherwise exact."""
    P = unflatten(np.asarray(w, dtype=np.float64))
    if bf16:
        for name, shape in PARAM_SHAPES:
            P[name] = bf16_round(P[name]) if len(shape) == 2 else P[name].astype(np.float32).astype(np.float64)
    return P


def forward(w, feat, bf16=False):
    """Returns (o [n, 48], cache).  With bf16=True the weights, the inputs
    and every GEMM input activation are rounded to bfloat16 as the GPU
    stores them (arithmetic stays FP64)."""
    rd = bf16_round if bf16 else (lambda a: a)
    P = _params(w, bf16)
    g = feat["graph"]
    src, dst = g["src"], g["dst"]
    n = g["n"]
    xn, xe = rd(feat["xn"]), rd(feat["xe"])
    deg = np.diff(g["ptr"]).astype(np.float64)
    c = dict(xn=xn, xe=xe)
    h = _relu(xn @ P["Wn"] + P["bn"])
    ge = _relu(xe @ P["We"] + P["be"])
    c["h0"], c["g"] = h, ge
    hs = [h]
    for l in range(N_LAYERS):
        hb, gb = rd(h), rd(ge)
        xm = np.concatenate([hb[src], hb[dst], gb], axis=1)
        m = _relu(xm @ P[f"M{l}"] + P[f"c{l}"])
        a = np.zeros((n, H))
        np.add.at(a, src, m)
        a /= np.maximum(deg, 1)[:, None]
        xu = np.concatenate([hb, rd(a)], axis=1)
        t = _relu(xu @ P[f"U{l}"] + P[f"u{l}"])
        c[f"xm{l}"], c[f"m{l}"], c[f"xu{l}"], c[f"t{l}"] = xm, m, xu, t
        h = h + t
        hs.append(h)
    c["hs"] = hs
    hb = rd(h)
    c["hL"] = hb
    o = hb @ P["Wd"] + P["bd"]
    return o, c


def factor_from_output(o):
    """Lt [n, 9, 9] from the decoder output."""
    n = o.shape[0]
    Lt = np.zeros((n, 9, 9))
    idx = np.arange(9)
    Lt[:, idx, idx] = np.exp(o[:, :9])
    for q, (r, cc) in enumerate(TRIL):
        Lt[:, r, cc] = o[:, 9 + q]
    return Lt


def loss_and_dout(o, z, y):
    """loss and d loss / d o for probes z, y: [n_probes, n, 9]."""
    npb, n, _ = z.shape
    Lt = factor_from_output(o)
    B = Lt @ np.transpose(Lt, (0, 2, 1))
    scale = 1.0 / (npb * 9 * n)
    r = np.einsum("nij,pnj->pni", B, y) - z
    loss = scale * float((r * r).sum())
    G = 2.0 * scale * np.einsum("pni,pnj->nij", r, y)          # d loss / d B
    dLt = np.einsum("nij,njk->nik", G + np.transpose(G, (0, 2, 1)), Lt)
    do = np.zeros_like(o)
    idx = np.arange(9)
    do[:, :9] = dLt[:, idx, idx] * Lt[:, idx, idx]
    for q, (rr, cc) in enumerate(TRIL):
        do[:, 9 + q] = dLt[:, rr, cc]
    return loss, do


def backward(w, feat, cache, do, bf16=False, extra=None):
    """Gradient of the loss with respect to the flat parameter vector;
    extra: gradients from the factorised head (dh on the final node states,
    dg on the encoded edge features, and the head's own parameters)."""
    rd = bf16_round if bf16 else (lambda a: a)
    P = _params(w, bf16)
    g = feat["graph"]
    src, dst = g["src"], g["dst"]
    n = g["n"]
    grads = {name: np.zeros(shape) for name, shape in PARAM_SHAPES}
    deg = np.diff(g["ptr"]).astype(np.float64)
    dob = rd(do)
    grads["Wd"] = cache["hL"].T @ dob
    grads["bd"] = do.sum(axis=0)
    dh = dob @ P["Wd"].T
    dg = np.zeros_like(cache["g"])
    if extra is not None:
        dh = dh + extra["dh"]
        dg = dg + extra["dg"]
        for name in ("Wo1", "bo1", "Wo2", "bo2", "ao"):
            grads[name] = extra[name]
    for l in reversed(range(N_LAYERS)):
        t = cache[f"t{l}"]
        dt = rd(dh * (t > 0))
        grads[f"U{l}"] = cache[f"xu{l}"].T @ dt
        grads[f"u{l}"] = (dh * (t > 0)).sum(axis=0)
        dxu = dt @ P[f"U{l}"].T
        dh = dh + dxu[:, :H]
        da = dxu[:, H:]
        m = cache[f"m{l}"]
        dm_f = (da / np.maximum(deg, 1)[:, None])[src] * (m > 0)
        dm = rd(dm_f)
        grads[f"M{l}"] = cache[f"xm{l}"].T @ dm
        grads[f"c{l}"] = dm_f.sum(axis=0)
        dxm = dm @ P[f"M{l}"].T
        np.add.at(dh, src, dxm[:, :H])
        np.add.at(dh, dst, dxm[:, H:2 * H])
        dg = dg + dxm[:, 2 * H:]
    h0, ge = cache["h0"], cache["g"]
    dpre_n = dh * (h0 > 0)
    grads["Wn"] = cache["xn"].T @ rd(dpre_n)
    grads["bn"] = dpre_n.sum(axis=0)
    dpre_e = dg * (ge > 0)
    grads["We"] = cache["xe"].T @ rd(dpre_e)
    grads["be"] = dpre_e.sum(axis=0)
    return flatten(grads)


def loss_and_grad(w, feat, z, bf16=False):
    """z: Rademacher probes [n_probes, n, 9]; returns (loss, grad, o)."""
    y = np.stack([normalised_product(feat, zp) for zp in z])
    o, cache = forward(w, feat, bf16)
    loss, do = loss_and_dout(o, z, y)
    return loss, backward(w, feat, cache, do, bf16), o


def preconditioner(o, L):
    """P_i = L_i^-T Lt_i Lt_i^T L_i^-1."""
    Lt = factor_from_output(o)
    out = np.empty_like(L)
    for i in range(L.shape[0]):
        Li = np.linalg.inv(L[i])
        out[i] = Li.T @ (Lt[i] @ Lt[i].T) @ Li
    return out


# ---------------------------------------------------------------------------
# factorised head (FSAI-pattern correction of block-Jacobi)
# ---------------------------------------------------------------------------
#
# M^-1 = G^T G with G block-lower-triangular on the sets J_i (camera i and
# its kept lower neighbours, ascending, i last).  In block-Jacobi-normalised
# coordinates Ghat = G blockdiag(L): Ghat_ii = Lt_i from the node decoder
# (lower triangular, diagonal exp(.)), and for j in J_i, j < i,
#     Ghat_ij = reshape(Wo2^T relu(Wo1^T [h_i, h_j, g_ij] + bo1) + bo2)[:81]
#               - ao[:81] * A_ij
# (A_ij the normalised block of the directed edge i -> j).  A zero head and
# decoder give Ghat = I, G = blockdiag(L^-1): block-Jacobi.  Training
# minimises the Kaporin functional in the normalised space,
#     f = (1/(9n)) sum_i [ tr(Ghat_i Ahat[J_i, J_i] Ghat_i^T)
#                          - 2 sum_k log (Ghat_ii)_kk ],
# whose minimiser over this pattern is the exact FSAI factor.

def fsai_edges(feat, J):
    """FSAI edges (i, member b < last) in row order: (src, dst, edge index)."""
    g = feat["graph"]
    index = {(int(a), int(b)): e for e, (a, b) in enumerate(zip(g["src"], g["dst"]))}
    out = []
    for i, Ji in enumerate(J):
        for j in Ji[:-1]:
            out.append((i, j, index[(i, j)]))
    return out


def fsai_factor(w, feat, J, bf16=False):
    """Returns (Ghat rows: list of [m_i, 9, 9] blocks, cache)."""
    rd = bf16_round if bf16 else (lambda a: a)
    o, cache = forward(w, feat, bf16)
    P = _params(w, bf16)
    A = feat["A"].astype(np.float32).astype(np.float64) if bf16 else feat["A"]
    hL = cache["hL"]
    gb = rd(cache["g"])
    fe = fsai_edges(feat, J)
    X = np.zeros((len(fe), 3 * H))
    for f, (i, j, e) in enumerate(fe):
        X[f] = np.concatenate([hL[i], hL[j], gb[e]])
    z1 = _relu(X @ P["Wo1"] + P["bo1"]) if len(fe) else np.zeros((0, HO))
    oe = rd(z1) @ P["Wo2"] + P["bo2"] if len(fe) else np.zeros((0, F_OFF))
    Lt = factor_from_output(o)
    rows, f = [], 0
    for i, Ji in enumerate(J):
        blocks = []
        for j in Ji[:-1]:
            e = fe[f][2]
            blocks.append(oe[f, :81].reshape(9, 9) - P["ao"][:81].reshape(9, 9) * A[e])
            f += 1
        blocks.append(Lt[i])
        rows.append(np.stack(blocks))
    cache.update(o=o, oe=oe, X=X, z1=z1, fe=fe, Aq=A)
    return rows, cache


def local_matrix(feat, Ji):
    """Ahat[J_i, J_i] (identity diagonal blocks)."""
    g = feat["graph"]
    index = {(int(a), int(b)): e for e, (a, b) in enumerate(zip(g["src"], g["dst"]))}
    m = len(Ji)
    M = np.zeros((9 * m, 9 * m))
    for a in range(m):
        for b in range(m):
            if a == b:
                M[9 * a:9 * a + 9, 9 * b:9 * b + 9] = np.eye(9)
            elif (Ji[a], Ji[b]) in index:
                M[9 * a:9 * a + 9, 9 * b:9 * b + 9] = feat["A"][index[(Ji[a], Ji[b])]]
    return M


def kaporin_loss(rows, feat, J):
    """f and d f / d Ghat (same layout as rows)."""
    n = len(J)
    N = 9.0 * n
    f = 0.0
    grads = []
    for Gi, Ji in zip(rows, J):
        m = len(Ji)
        Gr = np.concatenate(list(Gi), axis=1)            # 9 x 9m
        M = local_matrix(feat, Ji)
        Y = Gr @ M
        d = np.diag(Gi[-1])
        f += np.trace(Y @ Gr.T) - 2.0 * np.sum(np.log(d))
        dG = (2.0 / N) * Y
        dG[:, 9 * (m - 1):] -= (2.0 / N) * np.diag(1.0 / d)
        grads.append(dG.reshape(9, m, 9).transpose(1, 0, 2))
    return f / N, grads


def fsai_loss_and_grad(w, feat, J, bf16=False):
    """Kaporin loss of the factorised head and its gradient (flat)."""
    rd = bf16_round if bf16 else (lambda a: a)
    rows, cache = fsai_factor(w, feat, J, bf16)
    loss, dG = kaporin_loss(rows, feat, J)
    P = _params(w, bf16)
    o = cache["o"]
    n = o.shape[0]
    do = np.zeros_like(o)
    idx = np.arange(9)
    doe = np.zeros_like(cache["oe"])
    dao = np.zeros(F_OFF)
    A = cache["Aq"]
    f = 0
    for i, (Gi, Ji) in enumerate(zip(rows, J)):
        dGi = dG[i]
        dd = dGi[-1]
        do[i, :9] = dd[idx, idx] * Gi[-1][idx, idx]
        for q, (r, c) in enumerate(TRIL):
            do[i, 9 + q] = dd[r, c]
        for b in range(len(Ji) - 1):
            e = cache["fe"][f][2]
            doe[f, :81] = dGi[b].ravel()
            dao[:81] -= (dGi[b] * A[e]).ravel()
            f += 1
    doeb = rd(doe)
    X, z1 = cache["X"], cache["z1"]
    dz1 = (doeb @ P["Wo2"].T) * (z1 > 0)
    dz1b = rd(dz1)
    extra = dict(Wo2=rd(z1).T @ doeb, bo2=doe.sum(axis=0), ao=dao, Wo1=X.T @ dz1b, bo1=dz1.sum(axis=0))
    dX = dz1b @ P["Wo1"].T
    dh = np.zeros((n, H))
    dg = np.zeros_like(cache["g"])
    for f, (i, j, e) in enumerate(cache["fe"]):
        dh[i] += dX[f, :H]
        dh[j] += dX[f, H:2 * H]
        dg[e] += dX[f, 2 * H:]
    extra.update(dh=dh, dg=dg)
    return loss, backward(w, feat, cache, do, bf16, extra)


def fsai_preconditioner_factor(rows, J, L):
    """G rows in the original coordinates: G_ij = Ghat_ij L_j^-1."""
    out = []
    for Gi, Ji in zip(rows, J):
        out.append(np.stack([Gi[b] @ np.linalg.inv(L[j]) for b, j in enumerate(Ji)]))
    return out
