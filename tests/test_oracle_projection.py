"""Pins of the oracle's projection and Jacobians (CPU only).

- hand-derived projections with exactly known rotations (tests/golden);
- the rotation part against scipy's rotation-vector routine;
- Jacobians against central finite differences of the projection, at
  generic angles, near zero and near a half turn (Sec. 3.1: J is the
  Jacobian of the reprojection errors e).
"""
import json
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "projection_cases.json")


def _proj(cam, X):
    uv = orc.project(np.array([cam], float), np.array([X], float),
                     np.zeros(1, np.int32), np.zeros(1, np.int32))
    return uv[:, 0]


def test_golden_projections():
    cases = json.load(open(GOLDEN))["cases"]
    assert len(cases) >= 6
    for c in cases:
        got = _proj(c["cam"], c["X"])
        np.testing.assert_allclose(got, c["uv"], rtol=1e-12, atol=1e-12, err_msg=c["name"])


@pytest.mark.parametrize("theta", [0.0, 3e-9, 1e-6, 1e-3, 0.3, 1.0, 2.5, np.pi - 1e-3, np.pi])
def test_rotation_matches_scipy(theta):
    rng = np.random.default_rng(int(theta * 1000) + 7)
    for _ in range(20):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        w = axis * theta
        X = rng.normal(size=3)
        t = np.array([0.1, -0.2, 6.0])
        P = Rotation.from_rotvec(w).apply(X) + t
        cam = np.concatenate([w, t, [1.0, 0.0, 0.0]])
        got = _proj(cam, X)
        np.testing.assert_allclose(got, P[:2] / P[2], rtol=1e-13, atol=1e-15)


def _fd_jac(cam, X, h_rel=1e-6):
    x0 = np.concatenate([cam, X])
    J = np.zeros((2, 12))
    for k in range(12):
        h = h_rel * max(1.0, abs(x0[k]))
        xp = x0.copy(); xp[k] += h
        xm = x0.copy(); xm[k] -= h
        J[:, k] = (_proj(xp[:9], xp[9:]) - _proj(xm[:9], xm[9:])) / (2 * h)
    return J


@pytest.mark.parametrize("theta", [0.0, 5e-9, 1e-4, 0.7, 2.0, np.pi - 1e-4, np.pi])
def test_jacobian_finite_differences(theta):
    rng = np.random.default_rng(11)
    for _ in range(10):
        axis = rng.normal(size=3); axis /= np.linalg.norm(axis)
        cam = np.concatenate([axis * theta, rng.normal(0, 0.3, 3) + [0, 0, 8.0],
                              [rng.uniform(900, 1100), rng.uniform(-0.05, 0.05), rng.uniform(-0.01, 0.01)]])
        X = rng.normal(0, 1.0, 3)
        Pz = (Rotation.from_rotvec(cam[:3]).apply(X) + cam[3:6])[2]
        assert Pz > 1.0
        uv = np.zeros((2, 1))
        _, e, Jc, Jp = orc.linearize(cam[None], X[None], np.zeros(1, np.int32), np.zeros(1, np.int32), uv)
        J = np.concatenate([Jc[0], Jp[0]], axis=1)
        Jfd = _fd_jac(cam, X)
        scale = np.abs(J).max()
        np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-6 * scale)


def test_residual_zero_at_truth_noise_free(tiny_scene):
    """Noise-free data: e = 0 at the true parameters (cost 1/2 sum|e|^2 = 0)."""
    s = tiny_scene
    uv = orc.project(s.cams_true, s.pts_true, s.obs_cam, s.obs_pt)
    F, e, _, _ = orc.linearize(s.cams_true, s.pts_true, s.obs_cam, s.obs_pt, uv)
    assert F == 0.0 and np.all(e == 0.0)
    uvn = orc.observations(s)
    F2, e2, _, _ = orc.linearize(s.cams_true, s.pts_true, s.obs_cam, s.obs_pt, uvn)
    np.testing.assert_allclose(e2.T, -s.noise, atol=1e-9)
    np.testing.assert_allclose(F2, 0.5 * (s.noise ** 2).sum(), rtol=1e-12)
