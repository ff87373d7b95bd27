"""GPU keypoint descriptor matching (Sec. IV-B) against the oracle.

The kernels form squared distances |a|^2 + |b|^2 - 2 a.b in FP64 (dot
products on the FP64 matrix cores); the oracle sums (a - b)^2 in FP64.  The
two agree to rounding, so the per-row distances d1, d2 must agree within a
bound derived from FP64 arithmetic, and every match decision that differs
must be a certified near-tie: the row's two nearest distances, a column's two
nearest, or the ratio test's two sides within twice that bound.  Exactly
equal distances (duplicate descriptors) must resolve to the lowest index on
both sides.  Covered: every pair of a 10-keyframe window of 500 synthetic
keypoints with 128-D descriptors (the paper's detector setting) in one call,
with and without the ratio test; descriptor lengths 32, 64, 256; ragged and
empty sets around the 64-row tiles; argument errors.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def exact_sq_dists(A, B):
    A = A.astype(np.float64)
    B = B.astype(np.float64)
    return ((A[:, None, :] - B[None, :, :]) ** 2).sum(axis=2)


def dist_tol(A, B):
    dim = A.shape[1]
    na2 = (A.astype(np.float64) ** 2).sum(1).max(initial=0.0)
    nb2 = (B.astype(np.float64) ** 2).sum(1).max(initial=0.0)
    return 16 * dim * 2.0 ** -53 * (na2 + nb2 + 2 * np.sqrt(na2 * nb2)) + 1e-300


def check_pair(A, B, gm, gd1, gd2, ratio):
    """Compare one pair's GPU results with the oracle; return the number of
    certified differing decisions."""
    om, od1, od2 = oracle.match_descriptors(A, B, ratio)
    tol = dist_tol(A, B)
    fin1, fin2 = np.isfinite(od1), np.isfinite(od2)
    assert np.array_equal(np.isfinite(gd1), fin1) and np.array_equal(np.isfinite(gd2), fin2)
    assert np.all(np.abs(gd1[fin1] - od1[fin1]) <= tol)
    assert np.all(np.abs(gd2[fin2] - od2[fin2]) <= tol)
    diff = np.flatnonzero(gm != om)
    if diff.size == 0:
        return 0
    D = exact_sq_dists(A, B)
    col_sorted = np.sort(D, axis=0)
    for a in diff:
        row = np.sort(D[a])
        row_tie = row.size > 1 and row[1] - row[0] <= 2 * tol
        cols = [b for b in (gm[a], om[a], int(D[a].argmin())) if b >= 0]
        col_tie = any(D.shape[0] > 1 and col_sorted[1, b] - col_sorted[0, b] <= 2 * tol for b in cols)
        ratio_tie = ratio < 1.0 and abs(od1[a] - ratio ** 2 * od2[a]) <= 2 * tol * (1 + ratio ** 2)
        assert row_tie or col_tie or ratio_tie, (a, gm[a], om[a], row[:2], tol)
    return diff.size


def run(sets, pairs, ratio):
    import torch
    from paper_2108_00516_amd import frontend
    off = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int32)
    desc = torch.from_numpy(np.ascontiguousarray(np.concatenate(sets, axis=0))).cuda()
    m, d1, d2 = frontend.match_descriptors(desc, off, pairs, ratio)
    torch.cuda.synchronize()
    m, d1, d2 = m.cpu().numpy(), d1.cpu().numpy(), d2.cpu().numpy()
    out, o = [], 0
    for a, b in pairs:
        n = len(sets[a])
        out.append((m[o:o + n], d1[o:o + n], d2[o:o + n]))
        o += n
    return out


def unit(rng, n, dim):
    x = rng.normal(size=(n, dim))
    return (x / np.maximum(np.linalg.norm(x, axis=1, keepdims=True), 1e-30)).astype(np.float32)


@pytest.mark.parametrize("ratio", [1.0, 0.8])
def test_window_all_pairs_match_oracle(ratio):
    """All 45 keyframe pairs of the 10-keyframe window (500 keypoints, 128-D)
    in one call, both directions of three of them as well."""
    g = synth.make_graph("P")
    kf = synth.make_keypoints(g, n=500, dim=128, seed=1)
    sets = [k.desc for k in kf]
    pairs = [(i, j) for i in range(len(sets)) for j in range(i + 1, len(sets))] + [(3, 0), (9, 4), (5, 5)]
    print(f"match: {len(pairs)} pairs of {len(sets)} sets x 500 x 128, ratio {ratio}", flush=True)
    res = run(sets, pairs, ratio)
    n_diff = 0
    for (a, b), (gm, gd1, gd2) in zip(pairs, res):
        n_diff += check_pair(sets[a], sets[b], gm, gd1, gd2, ratio)
    # the generator's landmark correspondences are recovered (clutter
    # keypoints have random descriptors and pair up by chance)
    gm01 = res[0][0]
    lm0, lm1 = kf[0].landmark, kf[1].landmark
    ok = [lm1[y] == lm0[x] for x, y in enumerate(gm01) if y >= 0 and lm0[x] >= 0 and lm1[y] >= 0]
    # (with the ratio test every mutual match between landmarks is right;
    # without it a landmark whose partner is hidden pairs with another)
    assert len(ok) > 100 and np.mean(ok) >= (0.99 if ratio < 1.0 else 0.9)
    assert n_diff <= 3


@pytest.mark.parametrize("dim", [32, 64, 256])
def test_ragged_sets_and_lengths(dim):
    rng = np.random.default_rng(dim)
    sizes = [1, 63, 64, 65, 130, 0, 17, 200]
    sets = [unit(rng, n, dim) for n in sizes]
    # true partners: noisy copies of set 4's rows in set 7
    sets[7][:100] = sets[4][:100] + rng.normal(scale=0.05 / np.sqrt(dim), size=(100, dim)).astype(np.float32)
    pairs = [(0, 7), (1, 2), (2, 3), (3, 4), (4, 7), (7, 4), (5, 6), (6, 5), (6, 0), (3, 3)]
    print(f"match: ragged sets {sizes}, dim {dim}", flush=True)
    for ratio in (1.0, 0.9):
        res = run(sets, pairs, ratio)
        for (a, b), (gm, gd1, gd2) in zip(pairs, res):
            assert gm.shape == (len(sets[a]),)
            assert check_pair(sets[a], sets[b], gm, gd1, gd2, ratio) <= 1
        # a set against itself: every row is its own mutual nearest neighbour
        gm33 = res[-1][0]
        assert np.array_equal(gm33, np.arange(len(sets[3])))


def test_equal_distances_take_the_lowest_index():
    rng = np.random.default_rng(11)
    B = unit(rng, 70, 128)
    B[66] = B[3]          # duplicates across the 64-row tiles of B
    B[40] = B[3]
    A = np.concatenate([B[[3, 10]], unit(rng, 80, 128)]).astype(np.float32)
    A[70] = A[0]          # a duplicate row of A: column 3's nearest is the lower row 0
    res = run([A, B], [(0, 1), (1, 0)], 1.0)
    (gm, gd1, gd2), (hm, _, _) = res
    om, od1, od2 = oracle.match_descriptors(A, B, 1.0)
    assert np.array_equal(gm, om)
    assert gm[0] == 3 and gm[1] == 10 and gm[70] == -1
    assert gd2[0] == gd1[0] and abs(gd1[0]) <= dist_tol(A, B)   # equal distances, zero to rounding
    assert hm[3] == 0 and hm[40] == -1 and hm[66] == -1


def test_argument_errors():
    import torch
    from paper_2108_00516_amd import frontend
    from paper_2108_00516_amd import _lib as L
    desc = torch.zeros((10, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(frontend.FrontendError, match="INVALID_ARG"):
        frontend.match_descriptors(desc[:, :100].contiguous(), [0, 5, 10], [(0, 1)])   # dim 100
    with pytest.raises(frontend.FrontendError, match="INVALID_ARG"):
        frontend.match_descriptors(desc, [0, 5, 10], [(0, 2)])                          # no set 2
    with pytest.raises(frontend.FrontendError, match="CAPACITY"):
        frontend.match_descriptors(desc, [0, 5, 10], [(0, 1)] * 97)                     # too many pairs
    with pytest.raises(frontend.FrontendError, match="INVALID_ARG"):
        frontend.match_descriptors(desc, [0, 5, 10], [(0, 1)], ratio=0.0)
    big = torch.zeros((4097, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(frontend.FrontendError, match="CAPACITY"):
        frontend.match_descriptors(big, [0, 4097], [(0, 0)])
    # host memory is refused (the ABI takes device pointers)
    import ctypes as C
    lib = L.load()
    host = np.zeros((10, 128), np.float32)
    match = torch.zeros(5, dtype=torch.int32, device="cuda")
    off = np.array([0, 5, 10], np.int32)
    pa = np.array([0], np.int32)
    pb = np.array([1], np.int32)
    rc = lib.pg_match_descriptors(host.ctypes.data_as(C.c_void_p), off.ctypes.data_as(C.c_void_p), 2, 128,
                                  pa.ctypes.data_as(C.c_void_p), pb.ctypes.data_as(C.c_void_p), 1, 1.0,
                                  C.c_void_p(match.data_ptr()), None, None, None)
    assert rc == L.PG_ERR_INVALID_ARG
