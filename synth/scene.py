"""Seeded synthetic keyframe windows shaped like the paper's tracking workloads.

This module only *makes inputs*: a tabletop-scale object (a union of random
ellipsoids) seen by a pinhole RGB-D camera along a smooth trajectory, its depth
maps and masks, ground-truth and perturbed initial poses, and sparse pixel
matches with a known outlier fraction.  It contains none of the pose-graph
method's arithmetic (no association, residual, Jacobian, reduction, solve or
SE(3) update); both the FP64 oracle and the GPU library consume what it makes.

Stand-in for the paper's RGB-D test videos (NOCS, YCBInEOAT; Sec. V-A), which
are not available: objects of 3-8 cm features at 0.4-0.8 m, 640x480 depth, a
window of keyframes with mutual overlap (the overlap criterion of Sec. IV-C).

Poses are object-to-camera: x_cam = R x_obj + t, 4x4 row-major float64.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
from scipy.spatial.transform import Rotation

# Named workload presets.  Camera intrinsics, sizes, match counts and outlier
# fractions of each window; 'seed' is the default scene seed.
PRESETS = {
    # tiny: 4 keyframes at 160x120
    "T": dict(n_frames=4, width=160, height=120, fx=150.0, fy=150.0, cx=80.0, cy=60.0,
              n_matches=50, outlier_frac=0.10, seed=0),
    # paper scale: 10 keyframes at 640x480 (the window size class of Sec. IV-C)
    "P": dict(n_frames=10, width=640, height=480, fx=615.0, fy=615.0, cx=320.0, cy=240.0,
              n_matches=200, outlier_frac=0.20, seed=1),
    # 20 keyframes at 640x480 (precision and learned-weighting workloads)
    "X": dict(n_frames=20, width=640, height=480, fx=615.0, fy=615.0, cx=320.0, cy=240.0,
              n_matches=200, outlier_frac=0.20, seed=2),
    "L": dict(n_frames=20, width=640, height=480, fx=615.0, fy=615.0, cx=320.0, cy=240.0,
              n_matches=200, outlier_frac=0.20, seed=2),
}

# resolutions mixed in the batched workload; intrinsics scale with width
BATCH_RESOLUTIONS = [(320, 240), (480, 360), (640, 480)]

DEPTH_NOISE_SIGMA = 0.001   # metres, added to object pixels only
VISIBLE_TOL = 0.002         # an inlier match's target pixel must see the point within 2 mm
OUTLIER_MIN_DIST = 0.02     # an outlier pair is >= 2 cm apart in the object frame
BACKGROUND_Z = 1.1          # a back wall behind the object (outside the mask)


@dataclasses.dataclass
class MatchSet:
    i: int
    j: int
    uv_i: np.ndarray     # (n,2) float32 pixel coordinates (u, v) in frame i
    uv_j: np.ndarray     # (n,2) float32 pixel coordinates in frame j
    inlier: np.ndarray   # (n,) bool, generator truth


@dataclasses.dataclass
class SynthGraph:
    name: str
    seed: int
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    depth: np.ndarray        # (N,H,W) float32, metres, noisy
    depth_clean: np.ndarray  # (N,H,W) float32, noise-free render
    mask: np.ndarray         # (N,H,W) uint8, 1 = object
    poses_gt: np.ndarray     # (N,4,4) float64
    poses_init: np.ndarray   # (N,4,4) float64 (node 0 = ground truth)
    fixed: np.ndarray        # (N,) int32, node 0 fixed
    matches: List[MatchSet]

    @property
    def n_frames(self) -> int:
        return int(self.depth.shape[0])

    @property
    def hw(self) -> int:
        return self.width * self.height


def _rot(rotvec) -> np.ndarray:
    return Rotation.from_rotvec(np.asarray(rotvec, dtype=np.float64)).as_matrix()


def _random_rotation(rng) -> np.ndarray:
    # uniform on SO(3) via a unit quaternion drawn from a 4-D Gaussian
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return Rotation.from_quat(q).as_matrix()


def _make_scene(rng, n_ellipsoids=5):
    """Object model: ellipsoids with semi-axes in [3, 8] cm, random orientation,
    centres within +-5 cm of the object origin."""
    ells = []
    for _ in range(n_ellipsoids):
        axes = rng.uniform(0.03, 0.08, size=3)
        Q = _random_rotation(rng)
        c = rng.uniform(-0.05, 0.05, size=3)
        ells.append((c, Q, axes))
    return ells


def _trajectory(rng, n_frames):
    """Smooth oscillating object motion in front of the camera.

    Frame 0 places the object origin at (0, 0, z0), z0 in [0.55, 0.65] m, with a
    random base orientation.  Later frames add a sinusoidal yaw/pitch (amplitudes
    <= 30 / 20 deg) and a <= 1 cm translation wiggle, so consecutive frames stay
    within 10 deg / 3 cm and every pair of the window keeps overlap.
    """
    z0 = rng.uniform(0.55, 0.65)
    R_base = _random_rotation(rng)
    a_yaw = np.deg2rad(rng.uniform(15.0, 30.0))
    a_pitch = np.deg2rad(rng.uniform(8.0, 20.0))
    w_yaw = rng.uniform(0.15, 0.22)
    w_pitch = rng.uniform(0.15, 0.22)
    ph_yaw, ph_pitch = rng.uniform(0, 2 * np.pi, size=2)
    a_t = rng.uniform(0.003, 0.01, size=3)
    w_t = rng.uniform(0.1, 0.3, size=3)
    ph_t = rng.uniform(0, 2 * np.pi, size=3)
    poses = np.zeros((n_frames, 4, 4))
    yaw0 = a_yaw * np.sin(ph_yaw)
    pitch0 = a_pitch * np.sin(ph_pitch)
    for k in range(n_frames):
        yaw = a_yaw * np.sin(w_yaw * k + ph_yaw) - yaw0
        pitch = a_pitch * np.sin(w_pitch * k + ph_pitch) - pitch0
        R_m = _rot([0.0, yaw, 0.0]) @ _rot([pitch, 0.0, 0.0])
        t = np.array([0.0, 0.0, z0]) + a_t * (np.sin(w_t * k + ph_t) - np.sin(ph_t))
        poses[k, :3, :3] = R_m @ R_base
        poses[k, :3, 3] = t
        poses[k, 3, 3] = 1.0
    # motion-bound check between consecutive frames
    for k in range(1, n_frames):
        dR = poses[k, :3, :3] @ poses[k - 1, :3, :3].T
        ang = np.linalg.norm(Rotation.from_matrix(dR).as_rotvec())
        dt = np.linalg.norm(poses[k, :3, 3] - poses[k - 1, :3, 3])
        assert ang <= np.deg2rad(10.0) + 1e-12 and dt <= 0.03 + 1e-12, (k, ang, dt)
    return poses


def _pixel_rays(width, height, fx, fy, cx, cy):
    u = np.arange(width, dtype=np.float64)
    v = np.arange(height, dtype=np.float64)
    uu, vv = np.meshgrid(u, v)
    return np.stack([(uu - cx) / fx, (vv - cy) / fy, np.ones_like(uu)], axis=-1)  # (H,W,3)


def render(ells, pose, width, height, fx, fy, cx, cy):
    """Ray-cast the ellipsoids seen at 'pose'.  Returns (depth (H,W) float64 with
    0 where no object is hit, object-hit mask (H,W) bool).  The ray of pixel
    (u,v) has unit z, so the hit distance along it is the depth."""
    rays = _pixel_rays(width, height, fx, fy, cx, cy).reshape(-1, 3)
    R, t = pose[:3, :3], pose[:3, 3]
    best = np.full(rays.shape[0], np.inf)
    for (c, Q, axes) in ells:
        c_cam = R @ c + t
        Q_cam = R @ Q
        D = (rays @ Q_cam) / axes          # ray direction in the unit-sphere frame
        C = (Q_cam.T @ c_cam) / axes       # centre in the unit-sphere frame
        a = np.einsum("ij,ij->i", D, D)
        b = -2.0 * (D @ C)
        cc = C @ C - 1.0
        disc = b * b - 4.0 * a * cc
        hit = disc > 0
        sq = np.sqrt(np.where(hit, disc, 0.0))
        t0 = (-b - sq) / (2.0 * a)
        t1 = (-b + sq) / (2.0 * a)
        tt = np.where(t0 > 1e-6, t0, np.where(t1 > 1e-6, t1, np.inf))
        tt = np.where(hit, tt, np.inf)
        best = np.minimum(best, tt)
    hitmask = np.isfinite(best)
    depth = np.where(hitmask, best, 0.0)
    return depth.reshape(height, width), hitmask.reshape(height, width)


def _project(X, fx, fy, cx, cy):
    return np.stack([fx * X[:, 0] / X[:, 2] + cx, fy * X[:, 1] / X[:, 2] + cy], axis=-1)


def _backproject(u, v, z, fx, fy, cx, cy):
    return np.stack([z * (u - cx) / fx, z * (v - cy) / fy, z], axis=-1)


def _make_matches(rng, g_depth_clean, g_mask, poses, i, j, n, outlier_frac, K):
    """Pixel matches between frames i and j: (1-o)*n true correspondences
    (visible surface points, located through the ground-truth poses) and o*n
    gross outliers (point pairs >= 2 cm apart on the object)."""
    fx, fy, cx, cy, width, height = K
    n_out = int(round(outlier_frac * n))
    n_in = n - n_out
    vi_idx = np.flatnonzero(g_mask[i].ravel())
    vj_idx = np.flatnonzero(g_mask[j].ravel())
    Ti, Tj = poses[i], poses[j]
    Tji = Tj @ np.linalg.inv(Ti)
    # candidate inliers
    u = (vi_idx % width).astype(np.float64)
    v = (vi_idx // width).astype(np.float64)
    z = g_depth_clean[i].ravel()[vi_idx].astype(np.float64)
    Xi = _backproject(u, v, z, fx, fy, cx, cy)
    Xj = Xi @ Tji[:3, :3].T + Tji[:3, 3]
    ok = Xj[:, 2] > 1e-6
    uvj = _project(np.where(ok[:, None], Xj, 1.0), fx, fy, cx, cy)
    pj = np.floor(uvj + 0.5).astype(np.int64)
    inb = ok & (pj[:, 0] >= 0) & (pj[:, 0] < width) & (pj[:, 1] >= 0) & (pj[:, 1] < height)
    pidx = np.where(inb, pj[:, 1] * width + pj[:, 0], 0)
    vis = inb & (g_mask[j].ravel()[pidx] > 0) & (
        np.abs(g_depth_clean[j].ravel()[pidx] - Xj[:, 2]) < VISIBLE_TOL)
    cand = np.flatnonzero(vis)
    take = rng.choice(cand, size=min(n_in, cand.size), replace=False) if cand.size else np.zeros(0, np.int64)
    take = np.sort(take)
    uv_i_in = np.stack([u[take], v[take]], axis=-1)
    uv_j_in = uvj[take]
    # outliers: random object pixel pairs far apart in the object frame
    out_i, out_j = [], []
    if vi_idx.size and vj_idx.size:
        zj_all = g_depth_clean[j].ravel()
        Ti_inv, Tj_inv = np.linalg.inv(Ti), np.linalg.inv(Tj)
        tries = 0
        while len(out_i) < n_out and tries < 100:
            tries += 1
            a = rng.choice(vi_idx, size=4 * n_out)
            b = rng.choice(vj_idx, size=4 * n_out)
            Xa = _backproject((a % width).astype(float), (a // width).astype(float),
                              g_depth_clean[i].ravel()[a], fx, fy, cx, cy)
            Xb = _backproject((b % width).astype(float), (b // width).astype(float),
                              zj_all[b], fx, fy, cx, cy)
            Oa = Xa @ Ti_inv[:3, :3].T + Ti_inv[:3, 3]
            Ob = Xb @ Tj_inv[:3, :3].T + Tj_inv[:3, 3]
            far = np.linalg.norm(Oa - Ob, axis=1) >= OUTLIER_MIN_DIST
            for k in np.flatnonzero(far):
                if len(out_i) >= n_out:
                    break
                out_i.append(a[k])
                out_j.append(b[k])
    out_i = np.asarray(out_i, dtype=np.int64)
    out_j = np.asarray(out_j, dtype=np.int64)
    uv_i_out = np.stack([(out_i % width), (out_i // width)], axis=-1).astype(np.float64)
    uv_j_out = np.stack([(out_j % width), (out_j // width)], axis=-1).astype(np.float64)
    uv_i_all = np.concatenate([uv_i_in.reshape(-1, 2), uv_i_out.reshape(-1, 2)], axis=0)
    uv_j_all = np.concatenate([uv_j_in.reshape(-1, 2), uv_j_out.reshape(-1, 2)], axis=0)
    inl = np.concatenate([np.ones(len(take), bool), np.zeros(len(out_i), bool)])
    perm = rng.permutation(inl.size)
    return MatchSet(i, j, uv_i_all[perm].astype(np.float32), uv_j_all[perm].astype(np.float32), inl[perm])


def perturb_pose(rng, T, max_rot_rad, max_trans_m):
    """Left-perturb T by a random rotation of angle <= max_rot about a random
    axis (about the camera origin) and a random translation of length <= max_trans."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = rng.uniform(0.0, max_rot_rad)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    dt = d * rng.uniform(0.0, max_trans_m)
    P = np.eye(4)
    P[:3, :3] = _rot(axis * ang)
    P[:3, 3] = dt
    return P @ T


def make_graph(preset: str = "T", seed: Optional[int] = None, *, n_frames=None, width=None, height=None,
               noise_sigma: float = DEPTH_NOISE_SIGMA, init_rot_deg: float = 1.0, init_trans_m: float = 0.005,
               n_matches=None, outlier_frac=None, background: bool = True, mask_dilate: int = 0) -> SynthGraph:
    """Build one seeded keyframe window.

    preset: 'T', 'P', 'X', 'L' (see PRESETS) or 'B<k>' for the k-th graph of the
    batched workload (node count in 4..20, resolution from BATCH_RESOLUTIONS).
    Keyword overrides change sizes without changing the recipe.
    mask_dilate > 0 grows each mask by that many pixels (a square structuring
    element): the grown band covers back-wall pixels, the segmentation leaks a
    real pipeline's masks have at object boundaries.  Matches are drawn from
    the true object masks either way.
    """
    if preset.startswith("B"):
        k = int(preset[1:]) if len(preset) > 1 else 0
        brng = np.random.default_rng([1000, k])
        W, H = BATCH_RESOLUTIONS[int(brng.integers(0, len(BATCH_RESOLUTIONS)))]
        s = W / 640.0
        p = dict(n_frames=int(brng.integers(4, 21)), width=W, height=H, fx=615.0 * s, fy=615.0 * s,
                 cx=W / 2.0, cy=H / 2.0, n_matches=200, outlier_frac=0.20, seed=100 + k)
    else:
        p = dict(PRESETS[preset])
    if seed is None:
        seed = p["seed"]
    if n_frames is not None:
        p["n_frames"] = n_frames
    if width is not None:
        s = width / p["width"]
        p.update(width=width, fx=p["fx"] * s, cx=p["cx"] * s)
    if height is not None:
        s = height / p["height"]
        p.update(height=height, fy=p["fy"] * s, cy=p["cy"] * s)
    if n_matches is not None:
        p["n_matches"] = n_matches
    if outlier_frac is not None:
        p["outlier_frac"] = outlier_frac
    N, W, H = p["n_frames"], p["width"], p["height"]
    fx, fy, cx, cy = p["fx"], p["fy"], p["cx"], p["cy"]
    rng = np.random.default_rng(seed)
    ells = _make_scene(rng)
    poses = _trajectory(rng, N)
    depth_clean = np.zeros((N, H, W), np.float64)
    mask = np.zeros((N, H, W), np.uint8)
    for k in range(N):
        d, m = render(ells, poses[k], W, H, fx, fy, cx, cy)
        depth_clean[k] = d
        mask[k] = m.astype(np.uint8)
    noise = rng.normal(0.0, noise_sigma, size=depth_clean.shape) if noise_sigma > 0 else 0.0
    depth = np.where(mask > 0, depth_clean + noise, 0.0)
    if background:
        # a back wall outside the object region; it carries depth but no mask
        depth = np.where(mask > 0, depth, BACKGROUND_Z)
    matches = []
    K = (fx, fy, cx, cy, W, H)
    for i in range(N):
        for j in range(i + 1, N):
            mrng = np.random.default_rng([seed, i, j])
            matches.append(_make_matches(mrng, depth_clean, mask, poses, i, j, p["n_matches"],
                                         p["outlier_frac"], K))
    if mask_dilate > 0:
        from scipy.ndimage import binary_dilation
        st = np.ones((2 * mask_dilate + 1, 2 * mask_dilate + 1), bool)
        mask = np.stack([binary_dilation(m > 0, structure=st) for m in mask]).astype(np.uint8)
    prng = np.random.default_rng([seed, 7777])
    init = poses.copy()
    for k in range(1, N):
        init[k] = perturb_pose(prng, poses[k], np.deg2rad(init_rot_deg), init_trans_m)
    fixed = np.zeros(N, np.int32)
    fixed[0] = 1
    return SynthGraph(name=preset, seed=seed, width=W, height=H, fx=fx, fy=fy, cx=cx, cy=cy,
                      depth=depth.astype(np.float32), depth_clean=depth_clean.astype(np.float32),
                      mask=mask, poses_gt=poses, poses_init=init, fixed=fixed, matches=matches)


def plane_frames(n_frames=2, width=64, height=48, fx=60.0, fy=60.0, cx=32.0, cy=24.0,
                 normal=(0.2, -0.1, -1.0), offset=0.6):
    """Depth of the plane {x : n.x = -offset} (n normalised, facing the camera)
    seen by every frame: an input whose normals are known exactly."""
    n = np.asarray(normal, dtype=np.float64)
    n /= np.linalg.norm(n)
    rays = _pixel_rays(width, height, fx, fy, cx, cy)
    denom = rays @ n
    z = -offset / denom
    depth = np.where(z > 0, z, 0.0)
    return np.broadcast_to(depth, (n_frames, height, width)).astype(np.float32).copy(), n


def ransac_samples(seed: int, n_matches: int, n_hyp: int, pair: int = 0) -> np.ndarray:
    """The random draws of RANSAC for one pair: n_hyp samples of three
    distinct match indices in [0, n_matches), (n_hyp, 3) int32, from a seeded
    generator (seed, pair).  Fewer than three matches give all -1 rows."""
    rng = np.random.default_rng([seed, pair, 7])
    out = np.full((n_hyp, 3), -1, np.int32)
    if n_matches < 3:
        return out
    # three distinct indices: i0 uniform, i1 != i0, i2 not in {i0, i1}
    i0 = rng.integers(0, n_matches, n_hyp)
    i1 = rng.integers(0, n_matches - 1, n_hyp)
    i1 = i1 + (i1 >= i0)
    i2 = rng.integers(0, n_matches - 2, n_hyp)
    lo, hi = np.minimum(i0, i1), np.maximum(i0, i1)
    i2 = i2 + (i2 >= lo)
    i2 = i2 + (i2 >= hi)
    out[:, 0], out[:, 1], out[:, 2] = i0, i1, i2
    return out


@dataclasses.dataclass
class KeypointFrame:
    uv: np.ndarray         # (n, 2) float32 pixel coordinates (u, v)
    desc: np.ndarray       # (n, dim) float32 unit descriptors
    landmark: np.ndarray   # (n,) int32 landmark id, -1 for a clutter keypoint


def make_keypoints(g: SynthGraph, n: int = 500, dim: int = 128, n_landmarks: int = 600,
                   clutter_frac: float = 0.3, desc_noise: float = 0.15, seed: int = 0) -> List[KeypointFrame]:
    """Keypoints with descriptors for every frame of a window, standing in for
    the learned detector's n = 500 keypoints and 128-D descriptors: landmarks
    are object surface points (drawn from frame 0's clean render and kept in
    the object frame); a frame's keypoints are the landmarks visible in it
    (projected at its ground-truth pose, depth-consistent), each with its
    landmark's random unit descriptor plus N(0, desc_noise^2 / dim) noise per
    component, renormalised, then clutter keypoints (random object pixels with
    random descriptors) up to clutter_frac of n; at most n per frame, in
    random order."""
    rng = np.random.default_rng([seed, 4242])
    K = (g.fx, g.fy, g.cx, g.cy, g.width, g.height)
    fx, fy, cx, cy, width, height = K
    # landmarks: object points of frame 0 (object frame)
    m0 = np.flatnonzero(g.mask[0].ravel())
    pick = rng.choice(m0, size=min(n_landmarks, m0.size), replace=False)
    u = (pick % width).astype(np.float64)
    v = (pick // width).astype(np.float64)
    X0 = _backproject(u, v, g.depth_clean[0].ravel()[pick].astype(np.float64), fx, fy, cx, cy)
    T0inv = np.linalg.inv(g.poses_gt[0])
    Lobj = X0 @ T0inv[:3, :3].T + T0inv[:3, 3]
    base = rng.normal(size=(len(Lobj), dim))
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    frames = []
    n_clutter = int(round(clutter_frac * n))
    for f in range(g.n_frames):
        T = g.poses_gt[f]
        Xc = Lobj @ T[:3, :3].T + T[:3, 3]
        uv = _project(np.where(Xc[:, 2:3] > 1e-6, Xc, 1.0), fx, fy, cx, cy)
        p = np.floor(uv + 0.5).astype(np.int64)
        inb = (Xc[:, 2] > 1e-6) & (p[:, 0] >= 1) & (p[:, 0] < width - 1) & (p[:, 1] >= 1) & (p[:, 1] < height - 1)
        idx = np.where(inb, p[:, 1] * width + p[:, 0], 0)
        vis = inb & (g.mask[f].ravel()[idx] > 0) & (np.abs(g.depth_clean[f].ravel()[idx] - Xc[:, 2]) < VISIBLE_TOL)
        lm = np.flatnonzero(vis)
        lm = lm[rng.permutation(lm.size)][:n - n_clutter]
        d = base[lm] + rng.normal(scale=desc_noise / np.sqrt(dim), size=(lm.size, dim))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        mf = np.flatnonzero(g.mask[f].ravel())
        cl = rng.choice(mf, size=min(n_clutter, mf.size), replace=False)
        cd = rng.normal(size=(cl.size, dim))
        cd /= np.linalg.norm(cd, axis=1, keepdims=True)
        uv_all = np.concatenate([uv[lm], np.stack([cl % width, cl // width], axis=-1).astype(np.float64)])
        d_all = np.concatenate([d, cd])
        ids = np.concatenate([lm, np.full(cl.size, -1)])
        perm = rng.permutation(ids.size)
        frames.append(KeypointFrame(uv_all[perm].astype(np.float32), d_all[perm].astype(np.float32),
                                    ids[perm].astype(np.int32)))
    return frames
