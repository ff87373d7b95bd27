"""Pins of the synthetic input generator (scene synthesis, not the method)."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from synth.scene import render, _make_scene


def test_sphere_on_axis_depth():
    # a sphere of radius r centred on the optical axis at distance c: depth c - r
    ells = [(np.zeros(3), np.eye(3), np.array([0.05, 0.05, 0.05]))]
    T = np.eye(4)
    T[2, 3] = 0.5
    d, m = render(ells, T, 41, 31, 100.0, 100.0, 20.0, 15.0)
    assert m[15, 20]
    assert abs(d[15, 20] - 0.45) < 1e-12
    assert not m[0, 0] and d[0, 0] == 0.0


def test_rendered_points_on_ellipsoids():
    rng = np.random.default_rng(3)
    ells = _make_scene(rng)
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec([0.2, -0.1, 0.3]).as_matrix()
    T[2, 3] = 0.6
    W, H, f = 80, 60, 90.0
    d, m = render(ells, T, W, H, f, f, W / 2, H / 2)
    vv, uu = np.nonzero(m)
    z = d[vv, uu]
    X = np.stack([z * (uu - W / 2) / f, z * (vv - H / 2) / f, z], axis=1)
    Xo = (X - T[:3, 3]) @ T[:3, :3]          # back to the object frame
    best = np.full(len(z), np.inf)
    for (c, Q, a) in ells:
        y = ((Xo - c) @ Q) / a
        best = np.minimum(best, np.abs(np.linalg.norm(y, axis=1) - 1.0))
    assert best.max() < 1e-9


@pytest.mark.parametrize("preset", ["T", "B3"])
def test_determinism_and_shapes(preset):
    a = synth.make_graph(preset)
    b = synth.make_graph(preset)
    assert np.array_equal(a.depth, b.depth) and np.array_equal(a.mask, b.mask)
    assert np.array_equal(a.poses_init, b.poses_init)
    for ma, mb in zip(a.matches, b.matches):
        assert np.array_equal(ma.uv_i, mb.uv_i) and np.array_equal(ma.uv_j, mb.uv_j)
    N = a.n_frames
    assert a.depth.shape == (N, a.height, a.width) and a.depth.dtype == np.float32
    assert len(a.matches) == N * (N - 1) // 2
    c = synth.make_graph(preset, seed=a.seed + 1)
    assert not np.array_equal(a.depth, c.depth)


@pytest.mark.parametrize("seed", range(5))
def test_motion_bounds_and_init(seed):
    g = synth.make_graph("T", seed=seed, n_frames=12)
    for k in range(1, g.n_frames):
        dR = g.poses_gt[k, :3, :3] @ g.poses_gt[k - 1, :3, :3].T
        assert np.linalg.norm(Rotation.from_matrix(dR).as_rotvec()) <= np.deg2rad(10) + 1e-12
        assert np.linalg.norm(g.poses_gt[k, :3, 3] - g.poses_gt[k - 1, :3, 3]) <= 0.03
    assert np.array_equal(g.poses_init[0], g.poses_gt[0])
    for k in range(1, g.n_frames):
        dR = g.poses_init[k, :3, :3] @ g.poses_gt[k, :3, :3].T
        assert np.linalg.norm(Rotation.from_matrix(dR).as_rotvec()) <= np.deg2rad(1.0) + 1e-12
    z = g.depth_clean[g.mask > 0]
    assert z.min() > 0.35 and z.max() < 0.85


def test_match_ratio_and_truth():
    g = synth.make_graph("T")
    for m in g.matches:
        assert len(m.uv_i) == 50
        assert m.inlier.sum() == 45
        # ground-truth object-frame distance of each pair
        Ti, Tj = g.poses_gt[m.i], g.poses_gt[m.j]
        def obj(f, uv, T):
            u, v = np.floor(uv[:, 0] + 0.5).astype(int), np.floor(uv[:, 1] + 0.5).astype(int)
            z = g.depth_clean[f, v, u].astype(np.float64)
            X = np.stack([z * (u - g.cx) / g.fx, z * (v - g.cy) / g.fy, z], 1)
            return (X - T[:3, 3]) @ T[:3, :3]
        d = np.linalg.norm(obj(m.i, m.uv_i, Ti) - obj(m.j, m.uv_j, Tj), axis=1)
        assert np.all(d[~m.inlier] >= 0.02)
        assert np.median(d[m.inlier]) < 0.003


def test_mask_and_background():
    g = synth.make_graph("T")
    assert np.all(g.depth[g.mask == 0] == np.float32(synth.scene.BACKGROUND_Z))
    noise = (g.depth - g.depth_clean)[g.mask > 0]
    assert 0.0007 < noise.std() < 0.0013
