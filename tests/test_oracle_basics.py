"""Oracle pins: SE(3) exponential, Huber, Cholesky, per-frame preprocessing.

Each check compares the oracle with something other than itself: a library
routine (matrix exponential, rotation vectors, dense solve), a closed form
(plane normals, exact back-projection) or a defining property.
"""
import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

import oracle
import synth


def twist_matrix(xi):
    v, w = xi[:3], xi[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    M[:3, 3] = v
    return M


@pytest.mark.parametrize("scale", [0.0, 1e-9, 1e-7, 1e-3, 0.3, 1.5, 3.0])
def test_se3_exp_matches_matrix_exponential(oracle_lib, scale):
    rng = np.random.default_rng(11)
    for _ in range(10):
        xi = rng.normal(size=6)
        xi[3:] *= scale / max(np.linalg.norm(xi[3:]), 1e-300)
        T = oracle.se3_exp(xi)
        assert np.allclose(T, scipy.linalg.expm(twist_matrix(xi)), atol=1e-13, rtol=0)
        assert np.allclose(T[:3, :3], Rotation.from_rotvec(xi[3:]).as_matrix(), atol=1e-14)


def test_huber_closed_form(oracle_lib):
    d = 0.005
    for s in [0.0, 0.001, 0.004999, 0.005, 0.0050001, 0.02, 1.0]:
        rho = oracle.huber_rho(s, d)
        expect = 0.5 * s * s if s <= d else d * (s - 0.5 * d)
        assert rho == pytest.approx(expect, rel=1e-15, abs=0)
        # weight is rho'(s)/s
        h = 1e-9
        if s > 2 * h and abs(s - d) > 2 * h:
            drho = (oracle.huber_rho(s + h, d) - oracle.huber_rho(s - h, d)) / (2 * h)
            assert oracle.huber_weight(s, d) == pytest.approx(drho / s, rel=1e-5)
    # C1 continuity at the threshold
    e = 1e-12
    assert abs(oracle.huber_rho(d - e, d) - oracle.huber_rho(d + e, d)) < 1e-13
    assert abs(oracle.huber_weight(d - e, d) - oracle.huber_weight(d + e, d)) < 1e-9


@pytest.mark.parametrize("n", [1, 6, 18, 54, 114])
def test_cholesky_matches_dense_solve(oracle_lib, n):
    rng = np.random.default_rng(n)
    M = rng.normal(size=(n, n))
    A = M @ M.T + n * np.eye(n)
    b = rng.normal(size=n)
    rc, x = oracle.cholesky_solve(A, b)
    assert rc == oracle.OK
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-12)


def test_cholesky_flags_singular(oracle_lib):
    A = np.diag([1.0, 1.0, 0.0])
    rc, _ = oracle.cholesky_solve(A, np.ones(3))
    assert rc == oracle.ERR_SINGULAR
    v = np.array([1.0, 2.0, 3.0])
    rc, _ = oracle.cholesky_solve(np.outer(v, v), np.ones(3))
    assert rc == oracle.ERR_SINGULAR


def _problem(depth, mask, fx=60.0, fy=60.0, cx=32.0, cy=24.0):
    return oracle.OracleProblem(depth, mask, fx, fy, cx, cy)


def test_backprojection_round_trip(oracle_lib):
    g = synth.make_graph("T")
    pb = oracle.OracleProblem.from_synth(g)
    V, Nn, code = pb.preprocess(1)
    vv, uu = np.nonzero(code & 1)
    X = V[vv, uu]
    u = g.fx * X[:, 0] / X[:, 2] + g.cx
    v = g.fy * X[:, 1] / X[:, 2] + g.cy
    assert np.abs(u - uu).max() < 1e-9 and np.abs(v - vv).max() < 1e-9
    assert np.array_equal(X[:, 2], g.depth[1, vv, uu].astype(np.float64))


def test_plane_normals_exact(oracle_lib):
    depth, n_true = synth.plane_frames(n_frames=1)
    mask = np.ones_like(depth, np.uint8)
    pb = _problem(depth, mask)
    V, Nn, code = pb.preprocess(0)
    inner = code[1:-1, 1:-1]
    assert np.all(inner == 3)
    assert np.all(code[0, :] == 1) and np.all(code[:, -1] == 1)   # border: depth but no normal
    err = np.abs(Nn[1:-1, 1:-1] - n_true).max()
    # back-projected FP32 depths lie on the plane to ~1e-7 relative
    assert err < 1e-5
    # the normal faces the camera
    assert np.all(np.einsum("hwk,hwk->hw", Nn[1:-1, 1:-1], V[1:-1, 1:-1]) < 0)


def test_plane_normals_exact_in_fp64_depth(oracle_lib):
    # depth exactly representable on the plane z = 0.5 (fronto-parallel)
    depth = np.full((1, 20, 30), 0.5, np.float32)
    mask = np.ones_like(depth, np.uint8)
    V, Nn, code = _problem(depth, mask, cx=15.0, cy=10.0).preprocess(0)
    assert np.array_equal(Nn[1:-1, 1:-1], np.broadcast_to([0.0, 0.0, -1.0], Nn[1:-1, 1:-1].shape))


def test_validity_rules(oracle_lib):
    depth = np.full((1, 12, 16), 0.5, np.float32)
    mask = np.ones_like(depth, np.uint8)
    depth[0, 3, 4] = np.nan
    depth[0, 6, 8] = np.inf
    depth[0, 8, 10] = 0.0
    depth[0, 9, 3] = -0.2
    mask[0, 2, 12] = 0
    _, _, code = _problem(depth, mask, cx=8.0, cy=6.0).preprocess(0)
    for (v, u) in [(3, 4), (6, 8), (8, 10), (9, 3), (2, 12)]:
        assert code[v, u] == 0
        # the four neighbours lose their normal
        for (dv, du) in [(0, 1), (0, -1), (1, 0), (-1, 0)]:
            if 0 < v + dv < 11 and 0 < u + du < 15:
                assert code[v + dv, u + du] & 2 == 0
    assert code[5, 5] == 3


def test_sphere_normal_error_bounded(oracle_lib):
    # central differences on a sphere: normal error O(h/R) for pixel footprint h
    W, H, f = 120, 90, 200.0
    ells = [(np.zeros(3), np.eye(3), np.full(3, 0.08))]
    T = np.eye(4)
    T[2, 3] = 0.5
    d, m = synth.render(ells, T, W, H, f, f, W / 2, H / 2)
    pb = _problem(d[None].astype(np.float32), m[None].astype(np.uint8), f, f, W / 2, H / 2)
    V, Nn, code = pb.preprocess(0)
    ok = code == 3
    n_true = V[ok] - np.array([0, 0, 0.5])
    n_true /= np.linalg.norm(n_true, axis=1, keepdims=True)
    cosang = np.einsum("ij,ij->i", Nn[ok], n_true)
    h = 0.42 / f  # pixel footprint at the sphere
    assert np.median(np.arccos(np.clip(cosang, -1, 1))) < 5 * h / 0.08
