"""CPU pins of the oracle's coarse registration by RANSAC (Sec. IV-B): the
least-squares rigid transform of a sample (Arun et al.) against NumPy's SVD
and exact recovery; every hypothesis score against a brute-force NumPy
re-implementation; the best hypothesis against exhaustive search over all
triples of a small match set; unusable samples; and, on a rendered window with
known poses, the registration recovering the ground-truth relative pose while
rejecting every injected outlier."""
import itertools

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth

DELTA = 0.005
ALPHA = np.deg2rad(45.0)


def numpy_arun(a, b):
    """R, t minimising sum |R b + t - a|^2 via numpy.linalg.svd (textbook
    closed form with the reflection correction)."""
    ca, cb = a.mean(0), b.mean(0)
    U, _, Vt = np.linalg.svd((a - ca).T @ (b - cb))
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt))])
    R = U @ D @ Vt
    return R, ca - R @ cb


@pytest.mark.parametrize("k", [3, 4, 7, 12])
def test_arun_matches_numpy_svd(oracle_lib, k):
    rng = np.random.default_rng(k)
    for trial in range(20):
        R = Rotation.random(random_state=100 * k + trial).as_matrix()
        t = rng.normal(scale=0.1, size=3)
        b = rng.normal(scale=0.05, size=(k, 3)) + [0, 0, 0.6]
        a = b @ R.T + t + rng.normal(scale=2e-3, size=(k, 3))
        rc, T = oracle.arun(a, b)
        assert rc == oracle.OK
        Rn, tn = numpy_arun(a, b)
        assert np.abs(T[:3, :3] - Rn).max() < 1e-12
        assert np.abs(T[:3, 3] - tn).max() < 1e-12
        assert np.allclose(T[3], [0, 0, 0, 1])
        assert np.linalg.det(T[:3, :3]) == pytest.approx(1.0, abs=1e-12)


def test_arun_exact_recovery_and_degenerate(oracle_lib):
    rng = np.random.default_rng(3)
    R = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    t = np.array([0.01, -0.02, 0.03])
    b = rng.normal(scale=0.05, size=(3, 3)) + [0, 0, 0.6]
    rc, T = oracle.arun(b @ R.T + t, b)
    assert rc == oracle.OK
    assert np.abs(T[:3, :3] - R).max() < 1e-13 and np.abs(T[:3, 3] - t).max() < 1e-13
    # collinear points leave the rotation about their line free
    line = np.outer([0.0, 0.5, 1.0], [0.02, 0.03, 0.01]) + [0, 0, 0.6]
    rc, _ = oracle.arun(line @ R.T + t, line)
    assert rc == oracle.ERR_SINGULAR


def geometry(rng, n, n_out):
    """n matched points with normals under a known transform; the last n_out
    are gross outliers (>= 2 cm off)."""
    R = Rotation.from_rotvec(rng.normal(scale=0.15, size=3)).as_matrix()
    t = rng.normal(scale=0.02, size=3)
    b = rng.uniform(-0.06, 0.06, size=(n, 3)) + [0, 0, 0.6]
    nb = rng.normal(size=(n, 3))
    nb /= np.linalg.norm(nb, axis=1, keepdims=True)
    a = b @ R.T + t + rng.normal(scale=1e-3, size=(n, 3))
    na = nb @ R.T + rng.normal(scale=0.05, size=(n, 3))
    na /= np.linalg.norm(na, axis=1, keepdims=True)
    if n_out:
        d = rng.normal(size=(n_out, 3))
        a[n - n_out:] += 0.02 * d / np.linalg.norm(d, axis=1, keepdims=True) + rng.normal(scale=0.02, size=(n_out, 3))
    return a, na, b, nb, R, t


def brute_score(a, na, b, nb, valid, sample):
    s = list(sample)
    if len(set(s)) < 3 or min(s) < 0 or max(s) >= len(a) or not all(valid[s]):
        return -1, None
    for P in (a[s], b[s]):
        if 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0])) < 1e-8:
            return -1, None
    R, t = numpy_arun(a[s], b[s])
    d = np.linalg.norm(b @ R.T + t - a, axis=1)
    c = np.sum((nb @ R.T) * na, axis=1)
    inl = valid & (d < DELTA) & (c > np.cos(ALPHA))
    return int(inl.sum()), inl


def test_scores_match_brute_force(oracle_lib):
    rng = np.random.default_rng(5)
    a, na, b, nb, _, _ = geometry(rng, 60, 25)
    valid = np.ones(60, bool)
    valid[[3, 17]] = False
    samples = synth.ransac_samples(1, 60, 300)
    samples[0] = [4, 4, 9]            # repeated index
    samples[1] = [3, 20, 30]          # an invalid match
    for smp in samples:
        s, T, inl = oracle.ransac_score(a, na, b, nb, valid, smp)
        sb, ib = brute_score(a, na, b, nb, valid, smp)
        assert s == sb, smp
        if s >= 0:
            assert np.array_equal(inl, ib)


def test_best_hypothesis_is_exhaustive_maximum(oracle_lib):
    """With every triple of a 9-match set as a sample, the oracle's best
    hypothesis is the first one with the largest brute-force score."""
    rng = np.random.default_rng(8)
    a, na, b, nb, _, _ = geometry(rng, 9, 4)
    valid = np.ones(9, bool)
    triples = np.array(list(itertools.combinations(range(9), 3)), np.int32)
    scores = [oracle.ransac_score(a, na, b, nb, valid, t)[0] for t in triples]
    brute = [brute_score(a, na, b, nb, valid, t)[0] for t in triples]
    assert scores == brute
    assert max(brute) == 5              # the five true matches agree with each other


def test_registration_recovers_relative_pose(oracle_lib):
    """On a rendered window, RANSAC over each pair's matches (50 % gross
    outliers) returns a transform within 3 deg of the ground-truth relative
    rotation that carries the object's points to within 5 mm of where the
    ground-truth relative pose T_i T_j^-1 puts them (a three-point fit at
    160x120 is a coarse estimate: 4 mm pixels, 1 mm noise), keeps no injected
    outlier and most true matches."""
    g = synth.make_graph("T", outlier_frac=0.5)
    pb = oracle.OracleProblem.from_synth(g)
    pairs = [(m.j, m.i) for m in g.matches] + [(m.i, m.j) for m in g.matches]
    uvi = [m.uv_j for m in g.matches] + [m.uv_i for m in g.matches]
    uvj = [m.uv_i for m in g.matches] + [m.uv_j for m in g.matches]
    truth = [m.inlier for m in g.matches] * 2
    samples = np.stack([synth.ransac_samples(9, len(u), 500, pair=q) for q, u in enumerate(uvi)])
    out = pb.ransac(pairs, uvi, uvj, samples)
    for q, (i, j) in enumerate(pairs):
        assert out["best"][q] >= 0
        Tgt = g.poses_gt[i] @ np.linalg.inv(g.poses_gt[j])
        r, _ = oracle.pose_error(out["T"][q], Tgt)
        inl = out["inliers"][q]
        a, _, b, _, valid = _pair_geometry(pb, g, pairs[q], uvi[q], uvj[q])
        sel = truth[q] & valid.astype(bool)
        moved = b[sel] @ out["T"][q][:3, :3].T + out["T"][q][:3, 3]
        want = b[sel] @ Tgt[:3, :3].T + Tgt[:3, 3]
        assert r < np.deg2rad(3.0), (q, r)
        assert np.sqrt(np.mean(np.sum((moved - want) ** 2, axis=1))) < 0.005, q
        assert not (inl & ~truth[q]).any()
        assert inl.sum() >= 0.6 * truth[q].sum()
    # the transform is the sample's own least-squares fit and the flags are its inliers
    q, h = 0, out["best"][0]
    s, T, inl = oracle.ransac_score(*_pair_geometry(pb, g, pairs[0], uvi[0], uvj[0]), samples[0][h])
    assert np.array_equal(T, out["T"][0]) and np.array_equal(inl, out["inliers"][0])


def _pair_geometry(pb, g, pair, uv_i, uv_j):
    i, j = pair
    Vi, Ni, ci = pb.preprocess(i)
    Vj, Nj, cj = pb.preprocess(j)
    pi = np.floor(uv_i.astype(np.float64) + 0.5).astype(int)
    pj = np.floor(uv_j.astype(np.float64) + 0.5).astype(int)
    ok = lambda p: (p[:, 0] >= 0) & (p[:, 0] < g.width) & (p[:, 1] >= 0) & (p[:, 1] < g.height)
    vi, vj = ok(pi), ok(pj)
    pi[~vi] = 0
    pj[~vj] = 0
    valid = vi & vj & (ci[pi[:, 1], pi[:, 0]] == 3) & (cj[pj[:, 1], pj[:, 0]] == 3)
    return (Vi[pi[:, 1], pi[:, 0]], Ni[pi[:, 1], pi[:, 0]], Vj[pj[:, 1], pj[:, 0]], Nj[pj[:, 1], pj[:, 0]],
            valid.astype(np.uint8))


def test_registration_without_usable_sample(oracle_lib):
    g = synth.make_graph("T")
    pb = oracle.OracleProblem.from_synth(g)
    m = g.matches[0]
    out = pb.ransac([(m.i, m.j)], [m.uv_i[:2]], [m.uv_j[:2]], np.full((1, 4, 3), -1))
    assert out["best"][0] == -1 and np.array_equal(out["T"][0], np.eye(4))
    assert not out["inliers"][0].any()
