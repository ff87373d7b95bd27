"""GPU coarse registration by RANSAC (Sec. IV-B) against the oracle.

Both sides lift each match to 3-D points at its nearest pixels (identical
FP64 points from the same FP32 depth) with normals (FP32 on the GPU, FP64 in
the oracle, within 1e-5) and fit every sampled hypothesis by Arun's method in
FP64 with their own SVD codes.  So hypothesis scores must agree except for
matches at the decision boundaries: a score may differ only by matches whose
oracle distance is within 1e-9 m of delta or whose normal cosine is within
5e-5 of cos(alpha) (certified one by one); the best hypothesis' transform
must agree within 1e-9 and its inlier flags exactly, except certified
boundary matches.  Covered: every match set of the 4-keyframe (50 % gross
outliers) and 10-keyframe windows in both orientations, 300 hypotheses per
pair (a ragged last block of 64), the relative pose recovered within 5 deg
(a three-point fit on 1 mm depth noise is a coarse start: the oracle reaches
3.0 deg on one pair of the 10-keyframe window),
inliers installed as the pairs' feature matches and optimised against the
oracle, unusable samples, empty and tiny match sets, argument errors.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import check_normal_equations, gpu_decisions, gpu_graph, max_pose_diff, oracle_step

pytestmark = pytest.mark.gpu
DELTA = 0.005
ALPHA = float(np.deg2rad(45.0))
TOL_D = 1e-9
TOL_C = 5e-5


def pair_geometry(pb, g, pair, uv_i, uv_j):
    i, j = pair
    Vi, Ni, ci = pb.preprocess(i)
    Vj, Nj, cj = pb.preprocess(j)
    pi = np.floor(np.asarray(uv_i, np.float64) + 0.5).astype(int)
    pj = np.floor(np.asarray(uv_j, np.float64) + 0.5).astype(int)
    ok = lambda p: (p[:, 0] >= 0) & (p[:, 0] < g.width) & (p[:, 1] >= 0) & (p[:, 1] < g.height)
    vi, vj = ok(pi), ok(pj)
    pi[~vi] = 0
    pj[~vj] = 0
    valid = vi & vj & (ci[pi[:, 1], pi[:, 0]] == 3) & (cj[pj[:, 1], pj[:, 0]] == 3)
    return (Vi[pi[:, 1], pi[:, 0]], Ni[pi[:, 1], pi[:, 0]], Vj[pj[:, 1], pj[:, 0]], Nj[pj[:, 1], pj[:, 0]],
            valid.astype(np.uint8))


def boundary(T, geo):
    """Matches whose inlier decision under T sits at the delta / alpha boundary."""
    a, na, b, nb, valid = geo
    d = np.linalg.norm(b @ T[:3, :3].T + T[:3, 3] - a, axis=1)
    c = np.sum((nb @ T[:3, :3].T) * na, axis=1)
    return valid.astype(bool) & ((np.abs(d - DELTA) <= TOL_D) | (np.abs(c - np.cos(ALPHA)) <= TOL_C))


def window_pairs(g):
    pairs = [(m.j, m.i) for m in g.matches] + [(m.i, m.j) for m in g.matches]
    uvi = [m.uv_j for m in g.matches] + [m.uv_i for m in g.matches]
    uvj = [m.uv_i for m in g.matches] + [m.uv_j for m in g.matches]
    truth = [m.inlier for m in g.matches] * 2
    return pairs, uvi, uvj, truth


@pytest.mark.parametrize("name,outliers", [("T", 0.5), ("P", None)])
def test_ransac_matches_oracle(name, outliers):
    g = synth.make_graph(name, outlier_frac=outliers)
    pairs, uvi, uvj, truth = window_pairs(g)
    n_hyp = 300
    samples = np.stack([synth.ransac_samples(9, len(u), n_hyp, pair=q) for q, u in enumerate(uvi)])
    print(f"ransac {name}: {len(pairs)} pairs x {n_hyp} hypotheses", flush=True)
    pg = gpu_graph(g)
    out = pg.ransac(pairs, uvi, uvj, samples, DELTA, ALPHA, scores=True)
    pg.close()
    pb = oracle.OracleProblem.from_synth(g)
    ref = pb.ransac(pairs, uvi, uvj, samples, DELTA, ALPHA, scores=True)
    n_score_diff = 0
    for q, pair in enumerate(pairs):
        geo = pair_geometry(pb, g, pair, uvi[q], uvj[q])
        diff = np.flatnonzero(out["score"][q] != ref["score"][q])
        n_score_diff += diff.size
        for h in diff:
            s, T, _ = oracle.ransac_score(*geo, samples[q][h], DELTA, ALPHA)
            assert s >= 0 and out["score"][q][h] >= 0, (q, h)
            assert abs(int(out["score"][q][h]) - s) <= boundary(T, geo).sum(), (q, h)
        bg, bo = out["best"][q], ref["best"][q]
        if bg == bo:
            assert np.abs(out["T"][q] - ref["T"][q]).max() <= 1e-9, q
            flips = out["inliers"][q] != ref["inliers"][q]
            assert not (flips & ~boundary(ref["T"][q], geo)).any(), q
        else:
            # a near-equal score decided the best differently: both bests'
            # oracle scores within their boundary counts of each other
            sg, Tg, _ = oracle.ransac_score(*geo, samples[q][bg], DELTA, ALPHA)
            so, To, _ = oracle.ransac_score(*geo, samples[q][bo], DELTA, ALPHA)
            assert so - sg <= boundary(Tg, geo).sum() + boundary(To, geo).sum(), q
        # the registration recovers the ground-truth relative pose
        i, j = pair
        Tgt = g.poses_gt[i] @ np.linalg.inv(g.poses_gt[j])
        assert out["best"][q] >= 0
        assert oracle.pose_error(out["T"][q], Tgt)[0] < np.deg2rad(5.0), q   # a coarse 3-point fit
        assert not (out["inliers"][q] & ~truth[q]).any(), q
    assert n_score_diff <= 0.005 * len(pairs) * n_hyp


def test_installed_inliers_optimise_like_the_oracle():
    """install=True makes each pair's RANSAC inliers its feature matches (the
    C_ij of Eq. 2): the run that follows is bit for bit the run of a graph
    built with those matches, and every Gauss-Newton iteration agrees with the
    oracle on the GPU's association decisions (normal equations within 1e-5,
    the step within 1e-6).  End to end this window's 6th iteration meets an
    association decision at a near-tie that FP32 and FP64 take differently,
    so the 7-iteration poses are compared per iteration (as the paper-scale
    per-iteration test does)."""
    g = synth.make_graph("T", outlier_frac=0.3)
    fwd = [(m.i, m.j) for m in g.matches]
    uvi = [m.uv_i for m in g.matches]
    uvj = [m.uv_j for m in g.matches]
    samples = np.stack([synth.ransac_samples(4, len(u), 200, pair=q) for q, u in enumerate(uvi)])
    pg = gpu_graph(g)
    out = pg.ransac(fwd, uvi, uvj, samples, DELTA, ALPHA, install=True)
    st = pg.optimize()
    Pg = pg.poses
    pg.close()
    kept = [synth.MatchSet(m.i, m.j, m.uv_i[inl], m.uv_j[inl], m.inlier[inl])
            for m, inl in zip(g.matches, out["inliers"])]
    assert all(not (k.inlier == 0).any() for k in kept)
    g2 = synth.SynthGraph(**{**g.__dict__, "matches": kept})
    pg2 = gpu_graph(g2)
    st2 = pg2.optimize()
    assert np.array_equal(pg2.poses, Pg) and np.array_equal(st2["n_valid_f"], st["n_valid_f"])
    pg2.close()
    # per iteration on the GPU's decisions
    pg = gpu_graph(g, gn_iters=1)
    pg.ransac(fwd, uvi, uvj, samples, DELTA, ALPHA, install=True)
    pb = oracle.OracleProblem.from_synth(g2)
    P = pg.poses
    for it in range(7):
        lin = pb.linearize_given(P, gpu_decisions(pg, pb))
        H, gv, _ = pg.linearize()
        check_normal_equations(H, gv, lin)
        Q = oracle_step(lin, P, g.fixed)
        pg.optimize()
        P = pg.poses
        dr, dt = max_pose_diff(P, Q)
        assert dr <= 1e-6 and dt <= 1e-6, (it, dr, dt)
    pg.close()
    Po, so = oracle.OracleProblem.from_synth(g2).optimize(g.poses_init, 7)
    assert np.array_equal(st["n_valid_f"], so["n_valid_f"])
    dr, dt = max_pose_diff(Pg, Po)
    print(f"  installed inliers: {sum(len(k.uv_i) for k in kept)} matches; end to end vs oracle "
          f"{dr:.2e} rad {dt:.2e} m", flush=True)
    assert dr <= 1e-4 and dt <= 1e-4


def test_unusable_samples_and_small_sets():
    g = synth.make_graph("T")
    m = g.matches[0]
    pg = gpu_graph(g)
    pairs = [(m.i, m.j), (m.j, m.i), (m.i, m.j), (m.i, m.j)]
    uvi = [m.uv_i, m.uv_j, m.uv_i[:2], m.uv_i[:0]]
    uvj = [m.uv_j, m.uv_i, m.uv_j[:2], m.uv_j[:0]]
    samples = np.stack([synth.ransac_samples(1, len(u), 70, pair=q) for q, u in enumerate(uvi)])
    samples[0] = -1                    # no usable sample
    samples[1, :, 1] = samples[1, :, 0]  # every sample repeats a match
    out = pg.ransac(pairs, uvi, uvj, samples, DELTA, ALPHA, scores=True)
    for q in range(4):
        assert out["best"][q] == -1 and np.array_equal(out["T"][q], np.eye(4))
        assert (out["score"][q] == -1).all() and not out["inliers"][q].any()
    pg.close()


def test_argument_errors():
    from paper_2108_00516_amd import PoseGraphError
    g = synth.make_graph("T")
    m = g.matches[0]
    pg = gpu_graph(g)
    s = synth.ransac_samples(1, len(m.uv_i), 8).reshape(1, 8, 3)
    with pytest.raises(PoseGraphError, match="INVALID_ARG"):
        pg.ransac([(m.i, m.i)], [m.uv_i], [m.uv_j], s)
    with pytest.raises(PoseGraphError, match="INVALID_ARG"):
        pg.ransac([(m.i, 9)], [m.uv_i], [m.uv_j], s)
    with pytest.raises(PoseGraphError, match="CAPACITY"):
        pg.ransac([(m.i, m.j)], [m.uv_i], [m.uv_j], np.zeros((1, 8193, 3), np.int32))
    many = np.zeros((513, 2), np.float32)
    with pytest.raises(PoseGraphError, match="CAPACITY"):
        pg.ransac([(m.i, m.j)], [many], [many], s)
    with pytest.raises(PoseGraphError, match="INVALID_ARG"):
        pg.ransac([(m.i, m.j)], [m.uv_i], [m.uv_j], s, delta=0.0)
    pg.close()
