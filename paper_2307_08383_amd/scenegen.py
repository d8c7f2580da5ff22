"""Seeded synthetic bundle-adjustment scenes.

This module only draws random numbers and arranges them into a scene: true
camera and point parameters, which cameras see which point (the tracks),
per-observation pixel noise, and the perturbed starting parameters.  It holds
none of the bundle-adjustment arithmetic: it does not project points, so the
observed pixels are formed by whichever side consumes the scene
(``observed = projection(true parameters) + noise``), each with its own
projection routine.

The paper evaluates on aerial (UAV) blocks and on synthetic scenes with
N(0, 1) px noise (Sec. 7.1, Table 2); those datasets are not available, so the
scenes here reproduce their structure: nadir cameras on regular flight grids,
points spread over the covered ground, short tracks (mean ~4 observations per
point, between 2 and 12), a co-visibility graph with tens of neighbours per
camera, and Gaussian pixel noise.

Camera parameter layout (9 values): axis-angle rotation w (3), translation t
(3), focal length f, radial distortion k1, k2.  A world point X maps to the
camera frame as R(w) X + t and the camera looks along +z of its frame.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json

import numpy as np

N_CAM_PARAMS = 9


@dataclasses.dataclass
class Scene:
    name: str
    seed: int
    n_cams: int
    n_pts: int
    n_obs: int
    cams_true: np.ndarray      # float64 [n_cams][9]
    pts_true: np.ndarray       # float64 [n_pts][3]
    cams_init: np.ndarray      # float64 [n_cams][9]
    pts_init: np.ndarray       # float64 [n_pts][3]
    obs_cam: np.ndarray        # int32 [n_obs], sorted by (point, camera)
    obs_pt: np.ndarray         # int32 [n_obs]
    noise: np.ndarray          # float64 [2][n_obs] (u row, then v row)
    cam_fixed: np.ndarray      # uint8 [n_cams]
    lm_iterations: int
    pcg_tol: float
    stats: dict

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.cams_true, self.pts_true, self.cams_init, self.pts_init,
                  self.obs_cam, self.obs_pt, self.noise, self.cam_fixed):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


# --------------------------------------------------------------------------
# helpers (random draws and bookkeeping only)
# --------------------------------------------------------------------------

def _nadir_rotvecs(rng, n, tilt_sigma):
    """Axis-angle vectors of nadir-looking cameras with a small random tilt.

    The nadir attitude is the half turn about the world x axis (camera z
    points down); a small random rotation is composed on top so the angle
    never sits exactly at pi.  scipy's rotation class does the composition.
    """
    from scipy.spatial.transform import Rotation
    nadir = Rotation.from_rotvec(np.array([np.pi, 0.0, 0.0]))
    tilt = Rotation.from_rotvec(rng.normal(0.0, tilt_sigma, size=(n, 3)))
    rot = tilt * nadir
    return rot.as_rotvec(), rot


def _translations(rot, centres):
    """t = -R C, so that the camera centre C maps to the frame origin."""
    return -rot.apply(centres)


def _truncated_geometric(rng, n, lo, hi, mean):
    """Track lengths on [lo, hi] with P(t) ~ (1-p)^(t-lo), p set for `mean`."""
    ks = np.arange(lo, hi + 1)

    def mean_of(p):
        w = (1.0 - p) ** (ks - lo)
        return float((w * ks).sum() / w.sum())

    a, b = 1e-6, 1.0 - 1e-9
    for _ in range(200):
        m = 0.5 * (a + b)
        if mean_of(m) > mean:
            a = m
        else:
            b = m
    p = 0.5 * (a + b)
    w = (1.0 - p) ** (ks - lo)
    w /= w.sum()
    return rng.choice(ks, size=n, p=w).astype(np.int64), p


def _nearest_cams(centres_xy, pts_xy, t, k_pool, rng=None, choose_random=False,
                  chunk=1 << 20):
    """Per point, the t nearest camera centres in xy (or t drawn from the
    k_pool nearest).  Returns (obs_pt, obs_cam) sorted by (point, camera)."""
    from scipy.spatial import cKDTree
    tree = cKDTree(centres_xy)
    n = pts_xy.shape[0]
    obs_pt_parts, obs_cam_parts = [], []
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        _, idx = tree.query(pts_xy[s:e], k=k_pool, workers=-1)
        idx = idx.astype(np.int64)
        tt = t[s:e]
        if choose_random:
            keys = rng.random(size=idx.shape)
            order = np.argsort(keys, axis=1)
            idx = np.take_along_axis(idx, order, axis=1)
        mask = np.arange(k_pool)[None, :] < tt[:, None]
        sel = np.where(mask, idx, np.iinfo(np.int64).max)
        sel.sort(axis=1)
        rows = np.repeat(np.arange(s, e, dtype=np.int64), tt)
        obs_pt_parts.append(rows)
        obs_cam_parts.append(sel[np.arange(k_pool)[None, :] < tt[:, None]])
    return np.concatenate(obs_pt_parts), np.concatenate(obs_cam_parts)


def _covisibility_stats(n_cams, obs_pt, obs_cam, cam_fixed):
    """Neighbour counts of the co-visibility graph (pairs of cameras that
    share a point), used only to report the scene structure."""
    ptr = np.zeros(int(obs_pt.max()) + 2, dtype=np.int64)
    np.add.at(ptr, obs_pt + 1, 1)
    ptr = np.cumsum(ptr)
    t = np.diff(ptr)
    keys = []
    for tl in np.unique(t):
        pts = np.nonzero(t == tl)[0]
        base = ptr[pts]
        cams = obs_cam[base[:, None] + np.arange(tl)[None, :]]
        for a in range(tl):
            for b in range(a + 1, tl):
                ca, cb = cams[:, a], cams[:, b]
                keys.append(np.minimum(ca, cb) * n_cams + np.maximum(ca, cb))
    keys = np.unique(np.concatenate(keys)) if keys else np.zeros(0, np.int64)
    deg = np.zeros(n_cams, dtype=np.int64)
    np.add.at(deg, keys // n_cams, 1)
    np.add.at(deg, keys % n_cams, 1)
    n_triples = int((t * (t - 1) // 2).sum())
    return dict(mean_neighbours=float(deg.mean()), max_neighbours=int(deg.max()),
                n_pairs=int(keys.size), n_triples=int(n_triples),
                mean_track=float(t.mean()), max_track=int(t.max()))


def _assemble(name, seed, rng, centres, cam_fixed, pts, obs_pt, obs_cam,
              noise_sigma, lm_iterations, pcg_tol, tilt_sigma=0.02,
              with_stats=True):
    n_c = centres.shape[0]
    n_p = pts.shape[0]
    n_obs = obs_pt.size
    # intrinsics
    f = rng.uniform(950.0, 1050.0, size=n_c)
    k1 = rng.uniform(-0.05, 0.05, size=n_c)
    k2 = rng.uniform(-0.01, 0.01, size=n_c)
    w, rot = _nadir_rotvecs(rng, n_c, tilt_sigma)
    t = _translations(rot, centres)
    cams = np.empty((n_c, N_CAM_PARAMS))
    cams[:, 0:3] = w
    cams[:, 3:6] = t
    cams[:, 6] = f
    cams[:, 7] = k1
    cams[:, 8] = k2
    noise = rng.normal(0.0, 1.0, size=(2, n_obs)) * noise_sigma
    # start: each pose perturbed about its own centre (a small random
    # rotation, axis-angle components N(0, 0.01)) and its centre moved by
    # N(0, 0.05) per coordinate; intrinsics start at their true values
    from scipy.spatial.transform import Rotation
    rot_init = Rotation.from_rotvec(rng.normal(0.0, 0.01, size=(n_c, 3))) * rot
    centres_init = centres + rng.normal(0.0, 0.05, size=(n_c, 3))
    cams_init = cams.copy()
    cams_init[:, 0:3] = rot_init.as_rotvec()
    cams_init[:, 3:6] = _translations(rot_init, centres_init)
    fixed = cam_fixed.astype(bool)
    cams_init[fixed] = cams[fixed]
    pts_init = pts + rng.normal(0.0, 0.05, size=pts.shape)
    stats = dict(n_cams=n_c, n_pts=n_p, n_obs=int(n_obs), noise_sigma=noise_sigma,
                 n_fixed=int(fixed.sum()))
    if with_stats:
        stats.update(_covisibility_stats(n_c, obs_pt, obs_cam, cam_fixed))
    return Scene(name=name, seed=seed, n_cams=n_c, n_pts=n_p, n_obs=int(n_obs),
                 cams_true=cams, pts_true=pts, cams_init=cams_init, pts_init=pts_init,
                 obs_cam=obs_cam.astype(np.int32), obs_pt=obs_pt.astype(np.int32),
                 noise=noise, cam_fixed=cam_fixed.astype(np.uint8),
                 lm_iterations=lm_iterations, pcg_tol=pcg_tol, stats=stats)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def tiny_scene(seed=0, noise_sigma=0.5, n_grid=4, n_pts=500, t_lo=2, t_hi=6,
               with_stats=True):
    """16 cameras on a 4x4 grid at height 10 over [0,10]^2 looking down at
    500 points uniform in [0,10]x[0,10]x[0,1]; each point is seen by 2..6
    cameras drawn uniformly without replacement."""
    rng = np.random.default_rng(seed)
    g = (np.arange(n_grid) + 0.5) * (10.0 / n_grid)
    gx, gy = np.meshgrid(g, g, indexing="xy")
    centres = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 10.0)], axis=1)
    n_c = centres.shape[0]
    pts = np.stack([rng.uniform(0, 10, n_pts), rng.uniform(0, 10, n_pts),
                    rng.uniform(0, 1, n_pts)], axis=1)
    t = rng.integers(t_lo, t_hi + 1, size=n_pts)
    obs_pt, obs_cam = [], []
    for p in range(n_pts):
        sel = np.sort(rng.choice(n_c, size=t[p], replace=False))
        obs_pt.append(np.full(t[p], p))
        obs_cam.append(sel)
    obs_pt = np.concatenate(obs_pt)
    obs_cam = np.concatenate(obs_cam)
    return _assemble("tiny-16cam-500pt", seed, rng, centres, np.zeros(n_c, np.uint8),
                     pts, obs_pt, obs_cam, noise_sigma, lm_iterations=10,
                     pcg_tol=1e-6, with_stats=with_stats)


def aerial_grid_scene(seed=0, noise_sigma=0.5, nx=50, ny=40, n_pts=400_000,
                      spacing=1.0, altitude=2.5, relief=0.25, with_stats=True,
                      name=None, lm_iterations=20):
    """Nadir cameras on an nx x ny grid (60% overlap: footprint 2.5 grid
    steps at altitude 2.5 with image half-width 0.5 in normalised units),
    points uniform over the covered rectangle with relief in [0, 0.25], track
    length truncated-geometric on [2, 12] with mean 4, each point seen by the
    t nearest camera centres."""
    rng = np.random.default_rng(seed)
    xs = np.arange(nx) * spacing
    ys = np.arange(ny) * spacing
    gx, gy = np.meshgrid(xs, ys, indexing="xy")
    centres = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, altitude + 0.0)], axis=1)
    half = 0.5 * altitude  # half footprint: image half-width 0.5 times altitude
    pts = np.stack([rng.uniform(xs[0] - half, xs[-1] + half, n_pts),
                    rng.uniform(ys[0] - half, ys[-1] + half, n_pts),
                    rng.uniform(0.0, relief, n_pts)], axis=1)
    t, _ = _truncated_geometric(rng, n_pts, 2, 12, 4.0)
    obs_pt, obs_cam = _nearest_cams(centres[:, :2], pts[:, :2], t, 12)
    return _assemble(name or f"aerial-grid-{nx * ny}cam-{n_pts}pt", seed, rng, centres,
                     np.zeros(centres.shape[0], np.uint8), pts, obs_pt, obs_cam,
                     noise_sigma, lm_iterations=lm_iterations, pcg_tol=1e-6,
                     with_stats=with_stats)


def long_track_scene(seed=5, noise_sigma=0.5, nx=20, ny=15, n_pts=6000,
                     long_tracks=(12, 64, 65, 96, 200, 256, 257, 300), depth=20.0,
                     altitude=2.5, relief=0.25, with_stats=False):
    """The aerial grid plus a few distant points (depth units below the
    ground, near the grid centre, so every camera sees them within
    normalised radius ~0.65), point j seen by its long_tracks[j] nearest
    cameras: tracks longer than a 64-wide wave, up to every camera.  The
    distant points take random positions among the point indices."""
    rng = np.random.default_rng(seed)
    xs = np.arange(nx, dtype=np.float64)
    ys = np.arange(ny, dtype=np.float64)
    gx, gy = np.meshgrid(xs, ys, indexing="xy")
    centres = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, altitude)], axis=1)
    n_c = centres.shape[0]
    half = 0.5 * altitude
    near = np.stack([rng.uniform(xs[0] - half, xs[-1] + half, n_pts),
                     rng.uniform(ys[0] - half, ys[-1] + half, n_pts),
                     rng.uniform(0.0, relief, n_pts)], axis=1)
    t, _ = _truncated_geometric(rng, n_pts, 2, 12, 4.0)
    op_n, oc_n = _nearest_cams(centres[:, :2], near[:, :2], t, 12)
    lt = np.minimum(np.asarray(long_tracks, np.int64), n_c)
    n_l = lt.size
    far = np.stack([rng.uniform(0.4 * xs[-1], 0.6 * xs[-1], n_l),
                    rng.uniform(0.4 * ys[-1], 0.6 * ys[-1], n_l),
                    np.full(n_l, -depth)], axis=1)
    op_f, oc_f = _nearest_cams(centres[:, :2], far[:, :2], lt, int(lt.max()))
    # point ids: a random permutation of near and far points
    n_all = n_pts + n_l
    new_id = rng.permutation(n_all)
    pts = np.empty((n_all, 3))
    pts[new_id[:n_pts]] = near
    pts[new_id[n_pts:]] = far
    obs_pt = np.concatenate([new_id[op_n], new_id[n_pts + op_f]])
    obs_cam = np.concatenate([oc_n, oc_f])
    order = np.lexsort((obs_cam, obs_pt))
    return _assemble(f"long-tracks-{n_c}cam-{n_all}pt", seed, rng, centres, np.zeros(n_c, np.uint8), pts,
                     obs_pt[order], obs_cam[order], noise_sigma, lm_iterations=10, pcg_tol=1e-6,
                     with_stats=with_stats)


def strips_scene(seed=1, noise_sigma=0.5, n_strips=5, per_strip=3600, n_cross=2000,
                 n_pts=5_000_000, along=0.5, across=1.0, altitude=2.5, relief=0.25,
                 with_stats=True):
    """Flight strips along x (80% forward overlap: 0.5 steps for a 2.5-wide
    footprint, 60% side overlap: 1.0 between strips) plus cross strips along
    y, points uniform over the covered area, tracks as in the grid scene."""
    rng = np.random.default_rng(seed)
    cx = np.arange(per_strip) * along
    strips = [np.stack([cx, np.full(per_strip, s * across)], axis=1) for s in range(n_strips)]
    y_lo, y_hi = -1.0, (n_strips - 1) * across + 1.0
    n_per_cross = int(round((y_hi - y_lo) / along)) + 1
    n_cross_strips = max(1, n_cross // n_per_cross)
    cross = []
    xs_cross = np.linspace(cx[0], cx[-1], n_cross_strips)
    cy = np.linspace(y_lo, y_hi, n_per_cross)
    for x0 in xs_cross:
        cross.append(np.stack([np.full(n_per_cross, x0), cy], axis=1))
    cross = np.concatenate(cross)[:n_cross]
    if cross.shape[0] < n_cross:  # top up the last strip positions
        extra = n_cross - cross.shape[0]
        cross = np.concatenate([cross, np.stack([rng.uniform(cx[0], cx[-1], extra),
                                                 rng.uniform(y_lo, y_hi, extra)], axis=1)])
    xy = np.concatenate(strips + [cross])
    centres = np.concatenate([xy, np.full((xy.shape[0], 1), altitude)], axis=1)
    half = 0.5 * altitude
    pts = np.stack([rng.uniform(cx[0] - half, cx[-1] + half, n_pts),
                    rng.uniform(-half, (n_strips - 1) * across + half, n_pts),
                    rng.uniform(0.0, relief, n_pts)], axis=1)
    t, _ = _truncated_geometric(rng, n_pts, 2, 12, 4.0)
    obs_pt, obs_cam = _nearest_cams(centres[:, :2], pts[:, :2], t, 12)
    return _assemble(f"strips-{centres.shape[0]}cam-{n_pts}pt", seed, rng, centres,
                     np.zeros(centres.shape[0], np.uint8), pts, obs_pt, obs_cam,
                     noise_sigma, lm_iterations=10, pcg_tol=1e-6, with_stats=with_stats)


def partition_scene(seed=2, noise_sigma=0.5, nx=250, ny=240, ring=2, n_pts=25_000_000,
                    altitude=2.5, relief=0.25, k_pool=12, with_stats=False):
    """One partition of a larger block: an nx x ny grid of free cameras plus a
    ring of fixed cameras around it that belong to neighbouring partitions.
    Points lie over the partition; each point takes t cameras drawn among its
    k_pool nearest, so points near the edge are also seen by fixed cameras."""
    rng = np.random.default_rng(seed)
    xs = np.arange(-ring, nx + ring, dtype=np.float64)
    ys = np.arange(-ring, ny + ring, dtype=np.float64)
    gx, gy = np.meshgrid(xs, ys, indexing="xy")
    gx, gy = gx.ravel(), gy.ravel()
    inside = (gx >= 0) & (gx < nx) & (gy >= 0) & (gy < ny)
    order = np.concatenate([np.nonzero(inside)[0], np.nonzero(~inside)[0]])
    gx, gy, inside = gx[order], gy[order], inside[order]
    centres = np.stack([gx, gy, np.full(gx.size, altitude)], axis=1)
    cam_fixed = (~inside).astype(np.uint8)
    pts = np.stack([rng.uniform(-0.5, nx - 0.5, n_pts), rng.uniform(-0.5, ny - 0.5, n_pts),
                    rng.uniform(0.0, relief, n_pts)], axis=1)
    t, _ = _truncated_geometric(rng, n_pts, 2, 12, 4.0)
    obs_pt, obs_cam = _nearest_cams(centres[:, :2], pts[:, :2], t, k_pool, rng=rng,
                                    choose_random=True)
    return _assemble(f"partition-{int(inside.sum())}cam-{n_pts}pt", seed, rng, centres,
                     cam_fixed, pts, obs_pt, obs_cam, noise_sigma, lm_iterations=10,
                     pcg_tol=1e-6, with_stats=with_stats)


@dataclasses.dataclass
class SharedScene:
    """Images sharing the interior parameters of their physical camera:
    exterior [n_img][6] (axis-angle w, t), interior [n_phys][5] (f, cx, cy,
    k1, k2), img_cam [n_img] (physical camera of each image)."""
    name: str
    seed: int
    n_img: int
    n_phys: int
    n_pts: int
    n_obs: int
    img_cam: np.ndarray        # int32 [n_img]
    ext_true: np.ndarray       # float64 [n_img][6]
    intr_true: np.ndarray      # float64 [n_phys][5]
    pts_true: np.ndarray       # float64 [n_pts][3]
    ext_init: np.ndarray
    intr_init: np.ndarray
    pts_init: np.ndarray
    obs_img: np.ndarray        # int32 [n_obs]
    obs_pt: np.ndarray         # int32 [n_obs]
    noise: np.ndarray          # float64 [2][n_obs]
    img_fixed: np.ndarray      # uint8 [n_img]


def shared_intrinsics_scene(seed=0, nx=10, ny=8, n_pts=20_000, n_phys=4, noise_sigma=0.5, altitude=2.5,
                            relief=0.25, intr_sigma=0.0, long_tracks=(), depth=20.0):
    """The aerial grid (nadir images on an nx x ny grid, 60% overlap, tracks
    truncated-geometric on [2, 12] with mean 4, each point seen by its t
    nearest images) flown with n_phys physical cameras: image i is taken by
    camera i mod n_phys.  Interior: f ~ U(950, 1050) px, principal point
    (cx, cy) ~ U(-5, 5) px, k1 ~ U(-0.05, 0.05), k2 ~ U(-0.01, 0.01).  Start:
    poses perturbed as in the other scenes, interior parameters moved by
    N(0, intr_sigma) relative (0: at their true values).  long_tracks adds
    distant points as in long_track_scene (depth units below the ground near
    the grid centre, point j seen by its long_tracks[j] nearest images), at
    random point indices, drawn from a second generator so that the rest of
    the scene is that of the same seed without them."""
    rng = np.random.default_rng(seed)
    xs = np.arange(nx, dtype=np.float64)
    ys = np.arange(ny, dtype=np.float64)
    gx, gy = np.meshgrid(xs, ys, indexing="xy")
    centres = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, altitude)], axis=1)
    n_img = centres.shape[0]
    half = 0.5 * altitude
    pts = np.stack([rng.uniform(xs[0] - half, xs[-1] + half, n_pts),
                    rng.uniform(ys[0] - half, ys[-1] + half, n_pts),
                    rng.uniform(0.0, relief, n_pts)], axis=1)
    t, _ = _truncated_geometric(rng, n_pts, 2, 12, 4.0)
    obs_pt, obs_img = _nearest_cams(centres[:, :2], pts[:, :2], t, 12)
    intr = np.stack([rng.uniform(950.0, 1050.0, n_phys), rng.uniform(-5.0, 5.0, n_phys),
                     rng.uniform(-5.0, 5.0, n_phys), rng.uniform(-0.05, 0.05, n_phys),
                     rng.uniform(-0.01, 0.01, n_phys)], axis=1)
    w, rot = _nadir_rotvecs(rng, n_img, 0.02)
    ext = np.concatenate([w, _translations(rot, centres)], axis=1)
    noise = rng.normal(0.0, 1.0, size=(2, obs_pt.size)) * noise_sigma
    from scipy.spatial.transform import Rotation
    rot_init = Rotation.from_rotvec(rng.normal(0.0, 0.01, size=(n_img, 3))) * rot
    centres_init = centres + rng.normal(0.0, 0.05, size=(n_img, 3))
    ext_init = np.concatenate([rot_init.as_rotvec(), _translations(rot_init, centres_init)], axis=1)
    intr_init = intr * (1.0 + rng.normal(0.0, 1.0, size=intr.shape) * intr_sigma)
    pts_init = pts + rng.normal(0.0, 0.05, size=pts.shape)
    if len(long_tracks):
        r2 = np.random.default_rng(seed + 7919)
        lt = np.minimum(np.asarray(long_tracks, np.int64), n_img)
        far = np.stack([r2.uniform(0.4 * xs[-1], 0.6 * xs[-1], lt.size),
                        r2.uniform(0.4 * ys[-1], 0.6 * ys[-1], lt.size),
                        np.full(lt.size, -depth)], axis=1)
        op_f, oi_f = _nearest_cams(centres[:, :2], far[:, :2], lt, int(lt.max()))
        n_all = n_pts + lt.size
        new_id = r2.permutation(n_all)
        pts_all = np.empty((n_all, 3))
        init_all = np.empty((n_all, 3))
        pts_all[new_id[:n_pts]], pts_all[new_id[n_pts:]] = pts, far
        init_all[new_id[:n_pts]] = pts_init
        init_all[new_id[n_pts:]] = far + r2.normal(0.0, 0.05, size=far.shape)
        op = np.concatenate([new_id[obs_pt], new_id[n_pts + op_f]])
        oi = np.concatenate([obs_img, oi_f])
        nz = np.concatenate([noise, r2.normal(0.0, 1.0, size=(2, op_f.size)) * noise_sigma], axis=1)
        order = np.lexsort((oi, op))
        obs_pt, obs_img, noise = op[order], oi[order], nz[:, order]
        pts, pts_init, n_pts = pts_all, init_all, n_all
    return SharedScene(name=f"shared-{n_img}img-{n_phys}cam-{n_pts}pt", seed=seed, n_img=n_img, n_phys=n_phys,
                       n_pts=n_pts, n_obs=int(obs_pt.size), img_cam=(np.arange(n_img) % n_phys).astype(np.int32),
                       ext_true=ext, intr_true=intr, pts_true=pts, ext_init=ext_init, intr_init=intr_init,
                       pts_init=pts_init, obs_img=obs_img.astype(np.int32), obs_pt=obs_pt.astype(np.int32),
                       noise=noise, img_fixed=np.zeros(n_img, np.uint8))


WORKLOADS = {
    "tiny": tiny_scene,
    "aerial": aerial_grid_scene,
    "strips": strips_scene,
    "partition": partition_scene,
}


def make_scene(kind: str, **kw) -> Scene:
    return WORKLOADS[kind](**kw)


def shuffled(scene: Scene, seed: int = 123):
    """Same scene with the observation order permuted (tests that the
    consumer does not depend on the (point, camera) order)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(scene.n_obs)
    s = dataclasses.replace(scene, obs_cam=scene.obs_cam[perm].copy(),
                            obs_pt=scene.obs_pt[perm].copy(),
                            noise=scene.noise[:, perm].copy())
    return s, perm


def describe(scene: Scene) -> str:
    return json.dumps(dict(name=scene.name, seed=scene.seed, **scene.stats))
