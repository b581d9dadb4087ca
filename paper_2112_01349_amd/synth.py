"""Seeded synthetic bundle-adjustment problems.

This module is the shared input generator: it draws scenes, visibility and
noise and renders observations with a simulated pinhole sensor.  It holds no
part of the solver (no Rodrigues map, no Jacobian, no cost, no linear
algebra of the method).  Both the HIP path and the CPU oracle consume its
output unchanged.

Camera model used to render (the BAL convention that the paper's datasets
use, Sec. 6 dataset table): a camera with rotation matrix R, translation t,
focal f and radial terms k1, k2 maps a world point X to
    P = R X + t,  p = -(P_x, P_y) / P_z,
    u = f (1 + k1 |p|^2 + k2 |p|^4) p.
The rotation handed to the solver is the angle-axis vector of R, obtained
here by a quaternion log map (Shepperd's method) so that the rendered data
and the solver's own rotation route are independent.

Workload recipes (sizes and distributions from the paper's datasets and the
benchmark configurations):
  tiny   : 16 cameras on a ring of radius 10, 500 points in [-2,2]^3, each
           point seen by 2-6 uniformly chosen cameras, 1 px Gaussian noise.
  medium : 1,800 / 1.0M / 5.0M, stand-in for BAL Venice-1778 (Sec. 6 table).
  large  : 13,700 / 4.5M / 29M, stand-in for BAL Final-13682, 5% outliers.
  diff   : 1,000 / 200k / 1M, Huber workload for the gradient checks.
  stress : 20,000 / 10M / 60M, 5% outliers.
  synth20000 : the paper's synthesised production-like problem (Sec. 6,
           large synthesised dataset): 20,000 cameras evenly on a circle of
           radius 8, 80,000 points in a 0.2 x 0.2 x 0.06 slab at its centre,
           each seen by 1,000 distinct uniformly chosen cameras (80M
           observations, every point a long run).  synth_small is the same
           recipe at 400 / 1,600 / 480k for oracle-sized checks.
Zipf visibility: the number of views of a point follows a truncated power
law on [2, V_max] whose exponent is solved so that the mean equals N/n; the
cameras of a point are distinct and drawn with weights proportional to
rank^-1.2 over a seeded permutation of the camera ids.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Problem", "CONFIGS", "CIRCLE_CONFIGS", "generate", "point_chunk", "ring_rotation", "rotvec_from_matrix"]


@dataclass
class Problem:
    name: str
    cameras_true: np.ndarray   # [m, 9] f64: wx wy wz tx ty tz f k1 k2
    points_true: np.ndarray    # [n, 3] f64
    cameras0: np.ndarray       # [m, 9] f64, perturbed start
    points0: np.ndarray        # [n, 3] f64, perturbed start
    obs_camera: np.ndarray     # [N] int32
    obs_point: np.ndarray      # [N] int32
    obs_uv: np.ndarray         # [N, 2] f64 pixels
    outlier: np.ndarray        # [N] bool
    meta: dict = field(default_factory=dict)

    @property
    def num_cameras(self) -> int:
        return int(self.cameras0.shape[0])

    @property
    def num_points(self) -> int:
        return int(self.points0.shape[0])

    @property
    def num_obs(self) -> int:
        return int(self.obs_camera.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.cameras0, self.points0, self.obs_camera, self.obs_point, self.obs_uv):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


# name -> (m, n, N, V_max or None for the uniform 2..6 rule, scene half-width,
#          ring radius, outlier fraction)
CONFIGS = {
    "tiny":   dict(m=16, n=500, N=None, vmax=None, half=2.0, ring=10.0, outliers=0.0),
    "medium": dict(m=1800, n=1_000_000, N=5_000_000, vmax=40, half=50.0, ring=150.0, outliers=0.0),
    "large":  dict(m=13_700, n=4_500_000, N=29_000_000, vmax=60, half=50.0, ring=150.0, outliers=0.05),
    "diff":   dict(m=1000, n=200_000, N=1_000_000, vmax=40, half=50.0, ring=150.0, outliers=0.05),
    "stress": dict(m=20_000, n=10_000_000, N=60_000_000, vmax=80, half=50.0, ring=150.0, outliers=0.05),
}


# name -> circle recipe: cameras, points, views per point, circle radius
CIRCLE_CONFIGS = {
    "synth20000": dict(m=20_000, n=80_000, views=1_000, radius=8.0),
    "synth_small": dict(m=400, n=1_600, views=300, radius=8.0),
}


def ring_rotation(phi: float) -> np.ndarray:
    """Rotation (rows = camera axes in world frame) of a camera on the z=0 ring
    at angle phi whose optical axis (-z_cam) points at the origin."""
    c, s = math.cos(phi), math.sin(phi)
    z_cam = (c, s, 0.0)                 # C/|C|: the camera looks down -z
    x_cam = (-s, c, 0.0)                # world z cross z_cam (unit already)
    y_cam = (z_cam[1] * x_cam[2] - z_cam[2] * x_cam[1],
             z_cam[2] * x_cam[0] - z_cam[0] * x_cam[2],
             z_cam[0] * x_cam[1] - z_cam[1] * x_cam[0])
    return np.array([x_cam, y_cam, z_cam], dtype=np.float64)


def rotvec_from_matrix(R: np.ndarray) -> np.ndarray:
    """Angle-axis vector of a rotation matrix via a quaternion (Shepperd's
    choice of the largest pivot), robust at angles near pi."""
    m00, m01, m02 = R[0]
    m10, m11, m12 = R[1]
    m20, m21, m22 = R[2]
    tr = m00 + m11 + m22
    piv = max(tr, m00, m11, m22)
    if piv == tr:
        s = math.sqrt(1.0 + tr) * 2.0
        qw, qx, qy, qz = 0.25 * s, (m21 - m12) / s, (m02 - m20) / s, (m10 - m01) / s
    elif piv == m00:
        s = math.sqrt(1.0 + m00 - m11 - m22) * 2.0
        qw, qx, qy, qz = (m21 - m12) / s, 0.25 * s, (m01 + m10) / s, (m02 + m20) / s
    elif piv == m11:
        s = math.sqrt(1.0 + m11 - m00 - m22) * 2.0
        qw, qx, qy, qz = (m02 - m20) / s, (m01 + m10) / s, 0.25 * s, (m12 + m21) / s
    else:
        s = math.sqrt(1.0 + m22 - m00 - m11) * 2.0
        qw, qx, qy, qz = (m10 - m01) / s, (m02 + m20) / s, (m12 + m21) / s, 0.25 * s
    if qw < 0.0:
        qw, qx, qy, qz = -qw, -qx, -qy, -qz
    vn = math.sqrt(qx * qx + qy * qy + qz * qz)
    if vn == 0.0:
        return np.zeros(3)
    ang = 2.0 * math.atan2(vn, qw)
    return np.array([qx, qy, qz]) * (ang / vn)


def _apply_rows(R, X):
    """R[k] @ X[k] with plain elementwise products and sums (left to right),
    so the rendering is reproducible across CPUs."""
    out = np.empty_like(X)
    for a in range(3):
        out[:, a] = R[:, a, 0] * X[:, 0] + R[:, a, 1] * X[:, 1] + R[:, a, 2] * X[:, 2]
    return out


def _powers(base_from: int, base_to: int, expo: float) -> np.ndarray:
    """base**expo for integer bases, by scalar libm pow (identical on any CPU,
    unlike vectorised ufunc dispatch)."""
    return np.array([math.pow(float(b), expo) for b in range(base_from, base_to + 1)], dtype=np.float64)


def _power_law_exponent(mean: float, vmax: int) -> float:
    def mean_of(a):
        w = _powers(2, vmax, -a)
        num = 0.0
        den = 0.0
        for t, wt in enumerate(w):
            num += (t + 2) * wt
            den += wt
        return num / den

    lo, hi = 0.0, 10.0          # mean_of is decreasing in a
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_of(mid) > mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _views_per_point(rng, n, N, vmax, m):
    vmax = min(vmax, m)
    a = _power_law_exponent(N / n, vmax)
    k = np.arange(2, vmax + 1)
    w = _powers(2, vmax, -a)
    cdf = np.cumsum(w / math.fsum(w))
    cdf[-1] = 1.0
    views = k[np.searchsorted(cdf, rng.random(n), side="right")].astype(np.int64)
    # seeded fix-up: move the total onto N one view at a time, within bounds
    diff = int(N - views.sum())
    while diff != 0:
        cand = rng.integers(0, n, size=abs(diff) * 2 + 16)
        if diff > 0:
            cand = cand[views[cand] < vmax]
        else:
            cand = cand[views[cand] > 2]
        _, first = np.unique(cand, return_index=True)
        cand = cand[np.sort(first)][: abs(diff)]
        views[cand] += 1 if diff > 0 else -1
        diff = int(N - views.sum())
    return views, a


def _distinct_weighted(rng, views, weights):
    """For each point draw views[i] distinct ranks with probability ~ weights:
    draw with replacement, then redraw the repeats until every point's ranks
    are distinct."""
    n = views.shape[0]
    m = weights.shape[0]
    cdf = np.cumsum(weights / math.fsum(weights))
    cdf[-1] = 1.0
    N = int(views.sum())
    owner = np.repeat(np.arange(n, dtype=np.int64), views)
    rank = np.searchsorted(cdf, rng.random(N), side="right").astype(np.int64)
    active = np.arange(N, dtype=np.int64)       # positions still to check
    while active.size:
        key = owner[active] * m + rank[active]
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.size, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        redo = active[order[dup]]
        rank[redo] = np.searchsorted(cdf, rng.random(redo.size), side="right")
        # only points that had a repeat need checking again
        bad_pts = np.unique(owner[redo])
        sel = np.isin(owner[active], bad_pts)
        active = active[sel]
    return owner, rank


def _render(Rs, cams, pts, obs_camera, obs_point) -> np.ndarray:
    """Pixel coordinates of every observation under the sensor model."""
    N = obs_point.shape[0]
    uv = np.empty((N, 2), dtype=np.float64)
    chunk = 1 << 22
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        cj = obs_camera[s:e]
        X = pts[obs_point[s:e]]
        P = _apply_rows(Rs[cj], X) + cams[cj, 3:6]
        px = -P[:, 0] / P[:, 2]
        py = -P[:, 1] / P[:, 2]
        r2 = px * px + py * py
        d = 1.0 + cams[cj, 7] * r2 + cams[cj, 8] * r2 * r2
        fd = cams[cj, 6] * d
        uv[s:e, 0] = fd * px
        uv[s:e, 1] = fd * py
        assert np.all(P[:, 2] < 0.0), "point behind a camera"
    return uv


def _generate_circle(name: str, seed: int) -> Problem:
    """The synthesised recipe of Sec. 6.  The paper fixes the counts, the
    circle, the point box and the noise laws; where it is silent this takes:
    the circle in the z = 0 plane with every camera looking at its centre (as
    the ring rule of the other recipes), true intrinsics drawn as there
    (f ~ U[490, 510], k1 and k2 normal with standard deviation 1e-3), views drawn uniformly without
    replacement, observations rendered without pixel noise (the paper names
    none, so the optimum has zero cost), and the noise laws read as the
    perturbation of the start point: U(0, 0.01) added to every angle-axis
    and translation component, U(0, 0.5) to f, k1 and k2, U(-0.1, 0.1) to
    the x and y of every point."""
    cfg = CIRCLE_CONFIGS[name]
    m, n, views, radius = cfg["m"], cfg["n"], cfg["views"], cfg["radius"]
    rng = np.random.default_rng(seed)
    cams = np.zeros((m, 9), dtype=np.float64)
    Rs = np.zeros((m, 3, 3), dtype=np.float64)
    for j in range(m):
        phi = 2.0 * math.pi * (j + 0.5) / m
        R = ring_rotation(phi)
        C = np.array([radius * math.cos(phi), radius * math.sin(phi), 0.0])
        Rs[j] = R
        cams[j, 0:3] = rotvec_from_matrix(R)
        cams[j, 3:6] = -(R @ C)
    cams[:, 6] = rng.uniform(490.0, 510.0, size=m)
    cams[:, 7] = rng.normal(0.0, 1e-3, size=m)
    cams[:, 8] = rng.normal(0.0, 1e-3, size=m)
    pts = np.column_stack([rng.uniform(-0.1, 0.1, n), rng.uniform(-0.1, 0.1, n), rng.uniform(-0.03, 0.03, n)])
    obs_camera = np.empty(n * views, dtype=np.int32)
    for i in range(n):
        obs_camera[i * views:(i + 1) * views] = rng.choice(m, size=views, replace=False)
    obs_point = np.repeat(np.arange(n, dtype=np.int32), views)
    uv = _render(Rs, cams, pts, obs_camera, obs_point)
    cams0 = cams.copy()
    cams0[:, 0:6] += rng.uniform(0.0, 0.01, size=(m, 6))
    cams0[:, 6:9] += rng.uniform(0.0, 0.5, size=(m, 3))
    pts0 = pts.copy()
    pts0[:, 0:2] += rng.uniform(-0.1, 0.1, size=(n, 2))
    meta = dict(config=name, seed=seed, power_law_exponent=None, outlier_fraction=0.0)
    return Problem(name, cams, pts, cams0, pts0, obs_camera, obs_point, uv, np.zeros(n * views, dtype=bool), meta)


def generate(name: str, seed: int = 0, outliers: float | None = None) -> Problem:
    if name in CIRCLE_CONFIGS:
        assert outliers is None, "the synthesised recipe has no outliers"
        return _generate_circle(name, seed)
    cfg = CONFIGS[name]
    m, n, vmax, half, ring = cfg["m"], cfg["n"], cfg["vmax"], cfg["half"], cfg["ring"]
    out_frac = cfg["outliers"] if outliers is None else outliers
    rng = np.random.default_rng(seed)

    # cameras on a ring looking at the origin
    cams = np.zeros((m, 9), dtype=np.float64)
    Rs = np.zeros((m, 3, 3), dtype=np.float64)
    for j in range(m):
        phi = 2.0 * math.pi * (j + 0.5) / m
        R = ring_rotation(phi)
        C = np.array([ring * math.cos(phi), ring * math.sin(phi), 0.0])
        Rs[j] = R
        cams[j, 0:3] = rotvec_from_matrix(R)
        cams[j, 3:6] = -(R @ C)
    cams[:, 6] = rng.uniform(490.0, 510.0, size=m)
    cams[:, 7] = rng.normal(0.0, 1e-3, size=m)
    cams[:, 8] = rng.normal(0.0, 1e-3, size=m)

    pts = rng.uniform(-half, half, size=(n, 3))

    if vmax is None:   # uniform rule: 2..6 distinct uniformly chosen cameras
        views = rng.integers(2, 7, size=n)
        weights = np.ones(m)
        perm = np.arange(m)
        expo = None
    else:
        views, expo = _views_per_point(rng, n, cfg["N"], vmax, m)
        weights = _powers(1, m, -1.2)
        perm = rng.permutation(m)
    owner, rank = _distinct_weighted(rng, views, weights)
    obs_point = owner.astype(np.int32)
    obs_camera = perm[rank].astype(np.int32)
    N = obs_point.shape[0]

    # render with the sensor model (rotation matrix, not the angle-axis)
    uv = _render(Rs, cams, pts, obs_camera, obs_point)
    noise = rng.normal(0.0, 1.0, size=(N, 2))
    flag = np.zeros(N, dtype=bool)
    if out_frac > 0.0:
        flag = rng.random(N) < out_frac
        noise[flag] = rng.uniform(-50.0, 50.0, size=(int(flag.sum()), 2))
    uv_obs = uv + noise

    cams0 = cams * (1.0 + 0.01 * rng.normal(size=cams.shape))
    pts0 = pts * (1.0 + 0.01 * rng.normal(size=pts.shape))

    meta = dict(config=name, seed=seed, power_law_exponent=expo, outlier_fraction=out_frac)
    return Problem(name, cams, pts, cams0, pts0, obs_camera, obs_point, uv_obs, flag, meta)


def point_chunk(prob: Problem, k: int, K: int) -> Problem:
    """Chunk k of K of the edge partition made point-aligned: the points are
    cut, in index order, into K runs of about N/K observations each (a point
    is never split); the chunk keeps every camera and its own points,
    renumbered from 0, with their observations in the original order.  This
    is the share one of K GPUs would hold."""
    counts = np.bincount(prob.obs_point, minlength=prob.num_points)
    cum = np.concatenate([[0], np.cumsum(counts)])
    bounds = np.searchsorted(cum, np.arange(K + 1) * (prob.num_obs / K), side="left")
    bounds[0], bounds[-1] = 0, prob.num_points
    p0, p1 = int(bounds[k]), int(bounds[k + 1])
    sel = (prob.obs_point >= p0) & (prob.obs_point < p1)
    meta = dict(prob.meta, chunk=(k, K), points=(p0, p1))
    return Problem(f"{prob.name}_chunk{k}of{K}", prob.cameras_true, prob.points_true[p0:p1], prob.cameras0,
                   prob.points0[p0:p1], prob.obs_camera[sel], (prob.obs_point[sel] - p0).astype(np.int32),
                   prob.obs_uv[sel], prob.outlier[sel], meta)


def render_exact(prob: Problem) -> np.ndarray:
    """Noise-free rendering of the true scene (for zero-residual checks)."""
    m = prob.num_cameras
    ring = CIRCLE_CONFIGS[prob.name]["radius"] if prob.name in CIRCLE_CONFIGS else CONFIGS[prob.name]["ring"]
    Rs = np.stack([ring_rotation(2.0 * math.pi * (j + 0.5) / m) for j in range(m)])
    cj = prob.obs_camera
    X = prob.points_true[prob.obs_point]
    P = _apply_rows(Rs[cj], X) + prob.cameras_true[cj, 3:6]
    px = -P[:, 0] / P[:, 2]
    py = -P[:, 1] / P[:, 2]
    r2 = px * px + py * py
    fd = prob.cameras_true[cj, 6] * (1.0 + prob.cameras_true[cj, 7] * r2
                                     + prob.cameras_true[cj, 8] * r2 * r2)
    return np.stack([fd * px, fd * py], axis=1)
