"""Seeded synthetic bundle-adjustment scenes.

This module is the single source of inputs for both the oracle and the
GPU library.  It draws ground-truth cameras and points, decides which camera
sees which point, synthesises noisy pixel observations and perturbs the
ground truth into an initial estimate.  It holds none of the solver's
arithmetic (no residuals, Jacobians, normal equations or linear solves); the
only camera arithmetic here is the forward imaging used to synthesise pixels,
written on top of scipy's rotation primitives so that it shares no code with
either consumer.

Camera storage (one row of 10 float64 per camera), the convention every
consumer reads:
    [tx, ty, tz, qx, qy, qz, qw, f, k1, k2]
The pose maps world to camera: Y = R(q) X + t, with q a unit quaternion
stored scalar-last.  A point is in front of a camera when Y_z < 0 and its
pixel is f * D(s) * (-Y_x/Y_z, -Y_y/Y_z) with D(s) = 1 + k1 s + k2 s^2 and s
the squared norm of the normalised coordinates (the radially distorted
pinhole model of the paper's BAL benchmark, Sec. VI-A).

Workloads (scene sizes and structure follow the configurations of the
project; the paper's own BAL / 1DSfM datasets are not available, these
synthetic scenes stand in for them):
    0  ring: 16 cameras on a circle of radius 10 facing the origin,
       1,024 points in [-2,2]^3, 4 cameras per point, L2 loss, 10 LM iters.
    1  trajectory: 1,000 cameras on a smooth random walk, 200,000 points,
       power-law track lengths 2..30 (mean 5), Huber delta 1 px, 20 iters.
    2  laps: 10,000 cameras in 10 laps of a circuit, 2,000,000 points,
       track length 2+Poisson(2), 5% loop-closure re-assignments, 10 iters.
    3  differentiable layer: trajectory generator with 128 cameras, 20,000
       points, track 2+Poisson(3), observation weights U(0.5,1.5).
    4  preconditioner stream: scene `seed` of a stream, trajectory generator
       with U{200..2000} cameras, 10^U(4,5) points, track 2+Poisson(3) capped
       at 30 (about 5 observations per point), L2 loss.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = ["Scene", "make_scene", "image_points", "CONFIG_NAMES"]

CONFIG_NAMES = {
    0: "ring16_pts1024_obs4096",
    1: "traj1000_pts200k_obs1M_huber",
    2: "laps10000_pts2M_obs8M",
    3: "traj128_pts20k_obs100k_weighted",
    4: "stream_cams200-2000_pts1e4-1e5",
}


@dataclass
class Scene:
    cfg: int
    n_cams: int
    n_pts: int
    cam_idx: np.ndarray          # int32 [n_obs]
    pt_idx: np.ndarray           # int32 [n_obs]
    obs: np.ndarray              # float64 [n_obs, 2]
    obs_w: Optional[np.ndarray]  # float64 [n_obs] or None (all ones)
    cams_gt: np.ndarray          # float64 [n_cams, 10]
    pts_gt: np.ndarray           # float64 [n_pts, 3]
    cams0: np.ndarray            # float64 [n_cams, 10] initial estimate
    pts0: np.ndarray             # float64 [n_pts, 3]
    huber_delta: float = 0.0     # 0 => plain squared loss
    lm_iters: int = 10
    fixed_cams: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))

    @property
    def n_obs(self) -> int:
        return int(self.cam_idx.shape[0])

    def subset_observations(self, keep: np.ndarray) -> "Scene":
        """A copy with only the observations selected by `keep` (bool/index)."""
        return Scene(self.cfg, self.n_cams, self.n_pts, self.cam_idx[keep].copy(),
                     self.pt_idx[keep].copy(), self.obs[keep].copy(),
                     None if self.obs_w is None else self.obs_w[keep].copy(),
                     self.cams_gt, self.pts_gt, self.cams0, self.pts0,
                     self.huber_delta, self.lm_iters, self.fixed_cams)

    def permuted(self, perm: np.ndarray) -> "Scene":
        return self.subset_observations(perm)


# ----------------------------------------------------------------------------
# forward imaging (synthesis only)
# ----------------------------------------------------------------------------

def _to_camera(cams: np.ndarray, X: np.ndarray) -> np.ndarray:
    rot = Rotation.from_quat(cams[:, 3:7])
    return rot.apply(X) + cams[:, 0:3]


def image_points(cams: np.ndarray, X: np.ndarray):
    """Pixels of world points X[k] in cameras cams[k] (row-aligned arrays).

    Returns (pixels [n,2], camera-frame points [n,3])."""
    Y = _to_camera(cams, X)
    uv = -Y[:, 0:2] / Y[:, 2:3]
    s = np.einsum("ij,ij->i", uv, uv)
    dist = 1.0 + cams[:, 8] * s + cams[:, 9] * s * s
    return (cams[:, 7] * dist)[:, None] * uv, Y


def _look_rotations(view_dirs: np.ndarray) -> np.ndarray:
    """World->camera rotations whose camera looks along view_dirs (camera -z)."""
    z = -view_dirs / np.linalg.norm(view_dirs, axis=1, keepdims=True)
    up = np.array([0.0, 0.0, 1.0])
    x = np.cross(up[None, :], z)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=1)  # rows are the camera axes


def _cams_from(R: np.ndarray, C: np.ndarray, f: np.ndarray, k1: np.ndarray,
               k2: np.ndarray) -> np.ndarray:
    n = R.shape[0]
    cams = np.zeros((n, 10))
    cams[:, 0:3] = -np.einsum("nij,nj->ni", R, C)
    q = Rotation.from_matrix(R).as_quat()  # scalar-last
    q *= np.where(q[:, 3:4] < 0, -1.0, 1.0)
    cams[:, 3:7] = q
    cams[:, 7] = f
    cams[:, 8] = k1
    cams[:, 9] = k2
    return cams


def _visible(cams: np.ndarray, X: np.ndarray, max_uv: float = 0.7,
             max_z: float = -0.5) -> np.ndarray:
    return _visible_ids(_rot_table(cams), cams[:, 0:3], np.arange(cams.shape[0]), X,
                        max_uv, max_z)


def _rot_table(cams: np.ndarray) -> np.ndarray:
    return Rotation.from_quat(cams[:, 3:7]).as_matrix()


def _visible_ids(Rtab: np.ndarray, ttab: np.ndarray, ids: np.ndarray, X: np.ndarray,
                 max_uv: float = 0.7, max_z: float = -0.5) -> np.ndarray:
    Y = np.einsum("nij,nj->ni", Rtab[ids], X) + ttab[ids]
    with np.errstate(divide="ignore", invalid="ignore"):
        uv = -Y[:, 0:2] / Y[:, 2:3]
    return (Y[:, 2] <= max_z) & (np.abs(uv[:, 0]) <= max_uv) & (np.abs(uv[:, 1]) <= max_uv)


# ----------------------------------------------------------------------------
# perturbation of the ground truth into an initial estimate
# ----------------------------------------------------------------------------

def _perturb(rng, cams_gt, pts_gt, trans_scale, rot_rms=0.01, trans_rel=0.01,
             pt_sigma=0.05):
    """Rotation R <- Exp(phi) R with RMS |phi| = rot_rms; translation
    t <- t + N(0, (trans_rel * trans_scale)^2 / 3 I); points + N(0, pt_sigma^2 I);
    intrinsics are left at their true values."""
    n = cams_gt.shape[0]
    cams = cams_gt.copy()
    phi = rng.normal(size=(n, 3)) * (rot_rms / np.sqrt(3.0))
    rot = Rotation.from_rotvec(phi) * Rotation.from_quat(cams_gt[:, 3:7])
    q = rot.as_quat()
    q *= np.where(q[:, 3:4] < 0, -1.0, 1.0)
    cams[:, 3:7] = q
    sig = (trans_rel * trans_scale / np.sqrt(3.0))[:, None]
    cams[:, 0:3] += rng.normal(size=(n, 3)) * sig
    pts = pts_gt + rng.normal(size=pts_gt.shape) * pt_sigma
    return cams, pts


def _mean_depth_per_camera(cams, pts, cam_idx, pt_idx, n_cams):
    _, Y = image_points(cams[cam_idx], pts[pt_idx])
    depth = -Y[:, 2]
    s = np.bincount(cam_idx, weights=depth, minlength=n_cams)
    c = np.bincount(cam_idx, minlength=n_cams)
    out = np.where(c > 0, s / np.maximum(c, 1), np.median(depth))
    return out


# ----------------------------------------------------------------------------
# track builders
# ----------------------------------------------------------------------------

def _nearest_offsets(window: int) -> np.ndarray:
    off = [0]
    for k in range(1, window + 1):
        off += [-k, k]
    return np.array(off, dtype=np.int64)


def _tracks_nearest(rng, cams, n_pts, track_len, draw_point, window, wrap=None,
                    chunk=4096, max_rounds=200):
    """For every point pick its anchor camera plus the nearest-index cameras
    (|i - anchor| ascending, lower index first on ties) that see it, until the
    track has track_len[j] cameras.  Points whose candidates are too few are
    re-drawn.  `wrap` (period) makes the index distance cyclic inside blocks
    of that many cameras (laps)."""
    n_c = cams.shape[0]
    offs = _nearest_offsets(window)
    Rtab = _rot_table(cams)
    X = np.zeros((n_pts, 3))
    anchors = np.zeros(n_pts, np.int64)
    got_p, got_c = [], []
    todo = np.arange(n_pts)
    for _ in range(max_rounds):
        if todo.size == 0:
            break
        a, Xn = draw_point(rng, todo.size)
        anchors[todo] = a
        X[todo] = Xn
        failed = []
        for s in range(0, todo.size, chunk):
            idx = todo[s:s + chunk]
            aa = anchors[idx]
            if wrap is None:
                cand = aa[:, None] + offs[None, :]
                valid = (cand >= 0) & (cand < n_c)
            else:
                if offs.size > wrap:
                    raise ValueError("window larger than a lap")
                lap = aa // wrap
                ph = aa % wrap
                cand = lap[:, None] * wrap + (ph[:, None] + offs[None, :]) % wrap
                valid = np.ones(cand.shape, bool)
            cc = np.where(valid, cand, 0)
            vis = _visible_ids(Rtab, cams[:, 0:3], cc.ravel(),
                               np.repeat(X[idx], cand.shape[1], axis=0))
            vis = vis.reshape(cand.shape) & valid
            csum = np.cumsum(vis, axis=1)
            need = track_len[idx]
            ok = csum[:, -1] >= need
            take = vis & (csum <= need[:, None]) & ok[:, None]
            got_p.append(np.repeat(idx[ok], need[ok]))
            got_c.append(cand[take])
            failed.append(idx[~ok])
        todo = np.concatenate(failed) if failed else np.zeros(0, np.int64)
    if todo.size:
        raise RuntimeError(f"{todo.size} points found too few cameras")
    pid = np.concatenate(got_p)
    cid = np.concatenate(got_c)
    order = np.argsort(pid, kind="stable")
    return X, (pid[order].astype(np.int32), cid[order].astype(np.int32))


def _flatten_tracks(tracks):
    pid, cid = tracks
    return cid, pid


def _power_law_lengths(rng, n, lo=2, hi=30, alpha=1.966):
    t = np.arange(lo, hi + 1)
    p = t.astype(np.float64) ** (-alpha)
    p /= p.sum()
    return rng.choice(t, size=n, p=p)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def _ring(rng, n_cams, n_pts, per_pt):
    ang = 2.0 * np.pi * np.arange(n_cams) / n_cams
    C = 10.0 * np.stack([np.cos(ang), np.sin(ang), np.zeros(n_cams)], axis=1)
    R = _look_rotations(-C)
    k1 = rng.normal(size=n_cams) * 1e-3
    k2 = rng.normal(size=n_cams) * 1e-3
    cams = _cams_from(R, C, np.full(n_cams, 500.0), k1, k2)
    pts = rng.uniform(-2.0, 2.0, size=(n_pts, 3))
    cam_idx = np.concatenate([rng.choice(n_cams, size=per_pt, replace=False)
                              for _ in range(n_pts)]).astype(np.int32)
    pt_idx = np.repeat(np.arange(n_pts, dtype=np.int32), per_pt)
    return cams, pts, cam_idx, pt_idx


def _trajectory_cams(rng, n_cams):
    C = np.zeros((n_cams, 3))
    H = np.zeros((n_cams, 3))
    h = np.array([1.0, 0.0, 0.0])
    H[0] = h
    for i in range(1, n_cams):
        nz = rng.normal(size=3) * 0.3
        nz[2] *= 0.1
        h = h + nz
        h /= np.linalg.norm(h)
        H[i] = h
        C[i] = C[i - 1] + 0.5 * h
    C -= C.mean(axis=0)
    yaw = rng.uniform(-np.pi / 6, np.pi / 6, size=n_cams)
    cy, sy = np.cos(yaw), np.sin(yaw)
    d = np.stack([cy * H[:, 0] - sy * H[:, 1], sy * H[:, 0] + cy * H[:, 1], H[:, 2]], axis=1)
    R = _look_rotations(d)
    k1 = rng.normal(size=n_cams) * 1e-3
    k2 = rng.normal(size=n_cams) * 1e-3
    return _cams_from(R, C, np.full(n_cams, 500.0), k1, k2), R, C


def _anchored_point_drawer(R, C, n_cams, depth_lo, depth_hi):
    def draw(rng, n):
        a = rng.integers(0, n_cams, size=n)
        z = rng.uniform(depth_lo, depth_hi, size=n)
        uv = rng.uniform(-0.5, 0.5, size=(n, 2))
        Y = np.stack([z * uv[:, 0], z * uv[:, 1], -z], axis=1)
        X = np.einsum("nji,nj->ni", R[a], Y) + C[a]
        return a, X
    return draw


def _trajectory_scene(rng, n_cams, n_pts, track_len):
    cams, R, C = _trajectory_cams(rng, n_cams)
    draw = _anchored_point_drawer(R, C, n_cams, 4.0, 20.0)
    X, tracks = _tracks_nearest(rng, cams, n_pts, track_len, draw, window=50)
    cam_idx, pt_idx = _flatten_tracks(tracks)
    return cams, X, cam_idx, pt_idx


def _laps_scene(rng, n_cams, n_pts, per_lap=1000, loop_frac=0.05, radius=50.0, track_mean=2.0):
    if n_cams % per_lap:
        raise ValueError("n_cams must be a multiple of per_lap")
    n_laps = n_cams // per_lap
    i = np.arange(n_cams)
    lap = i // per_lap
    ph = 2.0 * np.pi * (i % per_lap) / per_lap
    r = radius + 0.5 * lap + rng.normal(size=n_cams) * 0.05
    C = np.stack([r * np.cos(ph), r * np.sin(ph), rng.normal(size=n_cams) * 0.05], axis=1)
    yaw = ph + rng.normal(size=n_cams) * 0.02
    d = np.stack([np.cos(yaw), np.sin(yaw), np.zeros(n_cams)], axis=1)
    R = _look_rotations(d)
    k1 = rng.normal(size=n_cams) * 1e-3
    k2 = rng.normal(size=n_cams) * 1e-3
    cams = _cams_from(R, C, np.full(n_cams, 500.0), k1, k2)
    track_len = np.minimum(2 + rng.poisson(track_mean, size=n_pts), min(30, per_lap // 3))
    draw = _anchored_point_drawer(R, C, n_cams, 5.0, 20.0)
    X, tracks = _tracks_nearest(rng, cams, n_pts, track_len, draw, window=20, wrap=per_lap)
    cam_idx, pt_idx = _flatten_tracks(tracks)
    if n_laps > 1 and loop_frac > 0:
        cam_idx = _loop_closures(rng, cams, X, cam_idx, pt_idx, per_lap, n_laps, loop_frac)
    return cams, X, cam_idx, pt_idx


def _loop_closures(rng, cams, X, cam_idx, pt_idx, per_lap, n_laps, frac, rounds=20):
    """Re-assign a uniformly chosen fraction of observations to a camera on a
    different lap at the same lap phase +-2 that sees the point and is not
    already in the point's track (re-drawn until it does, up to `rounds`)."""
    n_o = cam_idx.size
    cam_idx = cam_idx.copy()
    Rtab = _rot_table(cams)
    sel = rng.choice(n_o, size=int(round(frac * n_o)), replace=False)
    # existing (point, camera) pairs, to avoid duplicates
    key = pt_idx.astype(np.int64) * cams.shape[0] + cam_idx
    existing = set(key.tolist()) if n_o < 2_000_000 else None
    if existing is None:
        keys_sorted = np.sort(key)
    todo = sel
    for _ in range(rounds):
        if todo.size == 0:
            break
        c = cam_idx[todo]
        lap = c // per_lap
        dl = rng.integers(1, n_laps, size=todo.size)
        new_lap = (lap + dl) % n_laps
        dph = rng.integers(-2, 3, size=todo.size)
        new_c = new_lap * per_lap + (c % per_lap + dph) % per_lap
        vis = _visible_ids(Rtab, cams[:, 0:3], new_c, X[pt_idx[todo]])
        nk = pt_idx[todo].astype(np.int64) * cams.shape[0] + new_c
        if existing is not None:
            dup = np.array([k in existing for k in nk.tolist()], bool)
        else:
            pos = np.searchsorted(keys_sorted, nk)
            pos = np.minimum(pos, keys_sorted.size - 1)
            dup = keys_sorted[pos] == nk
        ok = vis & ~dup
        okk = todo[ok]
        cam_idx[okk] = new_c[ok]
        if existing is not None:
            existing.update(nk[ok].tolist())
        else:
            keys_sorted = np.sort(np.concatenate([keys_sorted, nk[ok]]))
        todo = todo[~ok]
    return cam_idx


def make_scene(cfg: int, seed: int = 0, noise_px: float = 1.0, perturb: bool = True,
               n_cams: Optional[int] = None, n_pts: Optional[int] = None,
               per_lap: Optional[int] = None, long_track: int = 0) -> Scene:
    """Build workload `cfg` with generator seed [cfg, seed].

    noise_px: standard deviation of the pixel noise per coordinate (0 gives
    noise-free observations).  perturb=False starts at the ground truth.
    n_cams / n_pts override the sizes (for small tests of a configuration's
    structure); per_lap sets the cameras per lap of the laps workload
    (default: 1000, or all cameras when fewer).  long_track (ring workload
    only): point 0 is seen by that many distinct cameras (every ring camera
    sees the whole point cube)."""
    rng = np.random.default_rng([cfg, seed])
    obs_w = None
    huber = 0.0
    fixed = np.zeros(0, np.int32)
    if cfg == 0:
        nc, npt = n_cams or 16, n_pts or 1024
        cams, pts, cam_idx, pt_idx = _ring(rng, nc, npt, per_pt=min(4, nc))
        if long_track:
            if long_track > nc:
                raise ValueError("long_track exceeds the number of cameras")
            keep = pt_idx != 0
            lt = np.sort(rng.choice(nc, size=long_track, replace=False)).astype(np.int32)
            cam_idx = np.concatenate([lt, cam_idx[keep]]).astype(np.int32)
            pt_idx = np.concatenate([np.zeros(long_track, np.int32), pt_idx[keep]]).astype(np.int32)
        iters = 10
    elif cfg == 1:
        nc, npt = n_cams or 1000, n_pts or 200_000
        tl = _power_law_lengths(rng, npt)
        tl = np.minimum(tl, max(2, min(101, nc // 3)))
        cams, pts, cam_idx, pt_idx = _trajectory_scene(rng, nc, npt, tl)
        huber, iters = 1.0, 20
    elif cfg == 2:
        nc, npt = n_cams or 10_000, n_pts or 2_000_000
        per_lap = per_lap or min(1000, nc)
        cams, pts, cam_idx, pt_idx = _laps_scene(rng, nc, npt, per_lap=per_lap)
        huber, iters = 1.0, 10
    elif cfg == 3:
        nc, npt = n_cams or 128, n_pts or 20_000
        tl = np.minimum(2 + rng.poisson(3.0, size=npt), max(2, min(30, nc // 3)))
        cams, pts, cam_idx, pt_idx = _trajectory_scene(rng, nc, npt, tl)
        iters = 50
        fixed = np.array([0, 1], np.int32)
    elif cfg == 4:
        # log-uniform sizes; laps of ~200 cameras with a random fraction
        # U(0, 0.1) of loop-closure observations; tracks 2 + Poisson(3)
        nc = n_cams or int(round(np.exp(rng.uniform(np.log(200), np.log(2000)))))
        npt = n_pts or int(round(np.exp(rng.uniform(np.log(1e4), np.log(1e5)))))
        laps = max(1, nc // 200)
        nc = (nc // laps) * laps
        frac = rng.uniform(0.0, 0.1)
        # circuit radius scaled so that cameras are spaced as in the large laps scene
        cams, pts, cam_idx, pt_idx = _laps_scene(rng, nc, npt, per_lap=nc // laps, loop_frac=frac,
                                                 radius=50.0 * (nc // laps) / 1000.0, track_mean=3.0)
        huber, iters = 1.0, 5
    else:
        raise ValueError(f"unknown configuration {cfg}")

    px, _ = image_points(cams[cam_idx], pts[pt_idx])
    obs = px + rng.normal(size=px.shape) * noise_px
    if cfg == 3:
        obs_w = rng.uniform(0.5, 1.5, size=cam_idx.size)

    if perturb:
        if cfg == 0:
            scale = np.linalg.norm(cams[:, 0:3], axis=1)
        else:
            scale = _mean_depth_per_camera(cams, pts, cam_idx, pt_idx, nc)
        cams0, pts0 = _perturb(rng, cams, pts, scale)
        if fixed.size:
            cams0[fixed] = cams[fixed]
    else:
        cams0, pts0 = cams.copy(), pts.copy()
    return Scene(cfg, nc, npt, cam_idx.astype(np.int32), pt_idx.astype(np.int32),
                 np.ascontiguousarray(obs), obs_w, cams, pts, cams0, pts0,
                 huber, iters, fixed)
