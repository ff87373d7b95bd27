"""Oracle pins: dense projective association (S2), residual Jacobians (S3/S4)
against central finite differences, and the normal equations' gradient against
the finite-difference gradient of the Huber energy with association frozen."""
import numpy as np
import pytest

import oracle
import synth


def _pose(rotvec=(0, 0, 0), t=(0, 0, 0)):
    from scipy.spatial.transform import Rotation
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(rotvec).as_matrix()
    T[:3, 3] = t
    return T


def test_identical_frames_map_to_themselves(oracle_lib):
    g = synth.make_graph("T", noise_sigma=0.0)
    depth = np.stack([g.depth[1], g.depth[1]])
    mask = np.stack([g.mask[1], g.mask[1]])
    pb = oracle.OracleProblem(depth, mask, g.fx, g.fy, g.cx, g.cy)
    poses = np.stack([g.poses_gt[1], g.poses_gt[1]])
    tgt, r, proj, gate = pb.associate(poses, 0, 1)
    _, _, code = pb.preprocess(0)
    src = np.flatnonzero(code.ravel() == 3)
    assert np.array_equal(tgt[src], src)
    assert np.all(tgt[code.ravel() != 3] == -1)
    assert np.abs(r[src]).max() < 1e-15
    assert np.abs(gate[src, 0]).max() < 1e-15


@pytest.mark.parametrize("k", [1, 3, -2])
def test_translated_plane_shifts_by_whole_pixels(oracle_lib, k):
    # fronto-parallel plane at z0: moving the object by k*z0/fx along x moves
    # its image by exactly k pixels
    W, H, f, z0 = 40, 30, 50.0, 0.5
    depth = np.full((2, H, W), z0, np.float32)
    mask = np.ones((2, H, W), np.uint8)
    pb = oracle.OracleProblem(depth, mask, f, f, W / 2, H / 2)
    poses = np.stack([_pose(t=(0, 0, 0)), _pose(t=(k * z0 / f, 0, 0))])
    tgt, r, proj, gate = pb.associate(poses, 0, 1)
    for v in range(1, H - 1):
        for u in range(1, W - 1):
            x = v * W + u
            if 1 <= u + k <= W - 2:
                assert tgt[x] == x + k
                assert abs(r[x]) < 1e-12
            elif 0 <= u + k <= W - 1:
                assert tgt[x] == -4      # lands on a border pixel without normal
            else:
                assert tgt[x] == -3      # outside the image


def test_gates(oracle_lib):
    W, H, f, z0 = 40, 30, 50.0, 0.5
    depth = np.full((2, H, W), z0, np.float32)
    mask = np.ones((2, H, W), np.uint8)
    pb = oracle.OracleProblem(depth, mask, f, f, W / 2, H / 2)
    inner = np.zeros((H, W), bool)
    inner[2:-2, 2:-2] = True
    inner = inner.ravel()
    # depth offset 0.5 cm passes the 1 cm distance gate, 1.5 cm fails it
    for dz, code in [(0.005, None), (0.015, -5)]:
        poses = np.stack([_pose(), _pose(t=(0, 0, dz))])
        tgt, r, _, gate = pb.associate(poses, 0, 1)
        if code is None:
            assert np.all(tgt[inner] >= 0)
            assert np.allclose(r[inner], -dz * 1.0, atol=1e-12) or np.allclose(r[inner], dz, atol=1e-12)
        else:
            assert np.all(tgt[inner] == code)
    # a 40 degree tilt between the two frames' normals fails the 30 degree gate
    depth2 = np.stack([depth[0], synth.plane_frames(1, W, H, f, f, W / 2, H / 2,
                                                    normal=(0, np.sin(np.deg2rad(40)), -np.cos(np.deg2rad(40))),
                                                    offset=z0 * np.cos(np.deg2rad(40)))[0][0]])  # both planes contain (0,0,z0)
    pb2 = oracle.OracleProblem(depth2, mask, f, f, W / 2, H / 2)
    tgt, _, _, gate = pb2.associate(np.stack([_pose(), _pose()]), 0, 1)
    sel = tgt != -1
    assert np.all(np.isin(tgt[sel], [-3, -4, -5, -6]))
    assert np.any(tgt[sel] == -6)
    c = gate[tgt == -6, 1]
    assert np.allclose(c, np.cos(np.deg2rad(40)), atol=1e-5)


def _perturbed(poses, node, k, h):
    P = poses.copy()
    xi = np.zeros(6)
    xi[k] = h
    P[node] = oracle.se3_exp(xi) @ P[node]
    return P


def test_dense_jacobian_finite_difference(oracle_lib):
    g = synth.make_graph("T")
    pb = oracle.OracleProblem.from_synth(g)
    poses = g.poses_init
    for (i, j) in [(0, 1), (2, 1), (3, 0)]:
        tgt, r, _, _ = pb.associate(poses, i, j)
        src = np.flatnonzero(tgt >= 0)[::7]
        t = tgt[src]
        r0, J = pb.dense_frozen(poses, i, j, src, t)
        assert np.allclose(r0, r[src], atol=1e-15)
        h = 1e-6
        for col in range(12):
            node, k = (i, col) if col < 6 else (j, col - 6)
            rp, _ = pb.dense_frozen(_perturbed(poses, node, k, h), i, j, src, t)
            rm, _ = pb.dense_frozen(_perturbed(poses, node, k, -h), i, j, src, t)
            fd = (rp - rm) / (2 * h)
            assert np.allclose(J[:, col], fd, rtol=1e-6, atol=1e-9), (i, j, col)


def test_feature_jacobian_finite_difference(oracle_lib):
    g = synth.make_graph("T")
    pb = oracle.OracleProblem.from_synth(g)
    poses = g.poses_init
    for s in [0, 3, 5]:
        i, j = pb.match_i[s], pb.match_j[s]
        for k in [0, 7, 19]:
            ok, e, J = pb.feature_eval(poses, s, k)
            assert ok
            h = 1e-6
            for col in range(12):
                node, kk = (i, col) if col < 6 else (j, col - 6)
                _, ep, _ = pb.feature_eval(_perturbed(poses, node, kk, h), s, k)
                _, em, _ = pb.feature_eval(_perturbed(poses, node, kk, -h), s, k)
                assert np.allclose(J[:, col], (ep - em) / (2 * h), rtol=1e-6, atol=1e-9)


def _frozen_energy(pb, poses, assoc, huber):
    """Huber energy of the dense term with the association frozen (S2 decisions
    taken once, at the linearisation poses)."""
    E = 0.0
    for (i, j), (src, tgt) in assoc.items():
        r, _ = pb.dense_frozen(poses, i, j, src, tgt)
        a = np.abs(r)
        E += np.where(a <= huber, 0.5 * a * a, huber * (a - 0.5 * huber)).sum()
    return E


def test_gradient_and_hessian_match_finite_differences(oracle_lib):
    # small graph, dense term only
    g = synth.make_graph("T", width=80, height=60, n_frames=3)
    prm = oracle.Params(lambda_f=0.0)
    pb = oracle.OracleProblem.from_synth(g, prm)
    poses = g.poses_init
    lin = pb.linearize(poses)
    N = g.n_frames
    assoc = {}
    for i in range(N):
        for j in range(N):
            if i != j:
                tgt, _, _, _ = pb.associate(poses, i, j)
                src = np.flatnonzero(tgt >= 0)
                assoc[(i, j)] = (src, tgt[src])
    E0 = _frozen_energy(pb, poses, assoc, prm.huber_g)
    assert E0 == pytest.approx(lin["energy_g"], rel=1e-12)
    h = 1e-6
    gfd = np.zeros(6 * N)
    for node in range(N):
        for k in range(6):
            Ep = _frozen_energy(pb, _perturbed(poses, node, k, h), assoc, prm.huber_g)
            Em = _frozen_energy(pb, _perturbed(poses, node, k, -h), assoc, prm.huber_g)
            gfd[6 * node + k] = (Ep - Em) / (2 * h)
    scale = lin["g_abs"].max()
    assert np.abs(lin["g"] - gfd).max() < 1e-6 * scale
    # Gauss-Newton Hessian: sum over residuals of w J J^T with J from finite differences
    Hfd = np.zeros((6 * N, 6 * N))
    for (i, j), (src, tgt) in assoc.items():
        r0, _ = pb.dense_frozen(poses, i, j, src, tgt)
        Jfd = np.zeros((len(src), 12))
        for col in range(12):
            node, k = (i, col) if col < 6 else (j, col - 6)
            rp, _ = pb.dense_frozen(_perturbed(poses, node, k, h), i, j, src, tgt)
            rm, _ = pb.dense_frozen(_perturbed(poses, node, k, -h), i, j, src, tgt)
            Jfd[:, col] = (rp - rm) / (2 * h)
        a = np.abs(r0)
        w = np.where(a <= prm.huber_g, 1.0, prm.huber_g / np.maximum(a, 1e-300))
        idx = np.r_[6 * i:6 * i + 6, 6 * j:6 * j + 6]
        Hfd[np.ix_(idx, idx)] += (Jfd * w[:, None]).T @ Jfd
    assert np.abs(lin["H"] - Hfd).max() < 1e-6 * np.abs(lin["H"]).max()
