"""CPU pins of the oracle's keypoint matching (Sec. IV-B: n keypoints with
128-D descriptors matched between frames): nearest neighbours against
scipy's pairwise distances, the mutual check as an inverse mapping, the ratio
test, equal distances resolved to the lowest index, empty sets, and on
synthetic keypoints the recovery of the generator's landmark
correspondences."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
import synth


def unit(rng, n, dim=128):
    x = rng.normal(size=(n, dim))
    return (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("na,nb,ratio", [(50, 70, 1.0), (120, 90, 0.9), (200, 200, 0.8)])
def test_matches_scipy_nearest_neighbours(oracle_lib, na, nb, ratio):
    rng = np.random.default_rng(na + nb)
    A, B = unit(rng, na), unit(rng, nb)
    # half of A are noisy copies of rows of B, so there are true mutual pairs
    src = rng.choice(nb, na // 2, replace=False)
    A[: na // 2] = B[src] + rng.normal(scale=0.02, size=(na // 2, 128)).astype(np.float32)
    m, d1, d2 = oracle.match_descriptors(A, B, ratio)
    D = cdist(A.astype(np.float64), B.astype(np.float64)) ** 2
    nn_a = D.argmin(axis=1)
    nn_b = D.argmin(axis=0)
    srt = np.sort(D, axis=1)
    assert np.allclose(d1, srt[:, 0], rtol=1e-12, atol=1e-14)
    assert np.allclose(d2, srt[:, 1], rtol=1e-12, atol=1e-14)
    want = np.where(nn_b[nn_a] == np.arange(na), nn_a, -1)
    if ratio < 1.0:
        want = np.where(srt[:, 0] < ratio ** 2 * srt[:, 1], want, -1)
    assert np.array_equal(m, want)
    assert (m[: na // 2] == src).mean() > 0.9


def test_mutual_matches_are_an_inverse_mapping(oracle_lib):
    rng = np.random.default_rng(3)
    A, B = unit(rng, 80), unit(rng, 60)
    B[:40] = A[10:50] + rng.normal(scale=0.03, size=(40, 128)).astype(np.float32)
    mab, _, _ = oracle.match_descriptors(A, B)
    mba, _, _ = oracle.match_descriptors(B, A)
    for a, b in enumerate(mab):
        if b >= 0:
            assert mba[b] == a
    for b, a in enumerate(mba):
        if a >= 0:
            assert mab[a] == b
    assert (mab >= 0).sum() == (mba >= 0).sum() >= 40


def test_equal_distances_take_the_lowest_index(oracle_lib):
    rng = np.random.default_rng(4)
    B = unit(rng, 10)
    B[7] = B[2]                     # a duplicate: A's nearest is the lower index 2
    A = B[[2, 5]].copy()
    m, d1, d2 = oracle.match_descriptors(A, B)
    assert m[0] == 2 and d1[0] == 0.0 and d2[0] == 0.0   # second nearest at the same distance
    assert m[1] == 5
    # with the ratio test an exact tie is not accepted (d1 < r^2 d2 fails)
    m, _, _ = oracle.match_descriptors(A, B, ratio=0.95)
    assert m[0] == -1 and m[1] == 5
    # duplicated rows of A: B[2]'s nearest of A is the lower index
    A2 = B[[2, 2, 5]].copy()
    m, _, _ = oracle.match_descriptors(A2, B)
    assert list(m) == [2, -1, 5]


def test_empty_sets(oracle_lib):
    rng = np.random.default_rng(5)
    A = unit(rng, 5)
    m, d1, _ = oracle.match_descriptors(A, np.zeros((0, 128), np.float32))
    assert np.all(m == -1) and np.all(np.isinf(d1))
    m, _, _ = oracle.match_descriptors(np.zeros((0, 128), np.float32), A)
    assert m.size == 0


def test_synthetic_keypoints_recover_landmarks(oracle_lib):
    g = synth.make_graph("T")
    kp = synth.make_keypoints(g, n=300, n_landmarks=400)
    for (i, j) in [(0, 1), (1, 3), (2, 0)]:
        a, b = kp[i], kp[j]
        m, _, _ = oracle.match_descriptors(a.desc, b.desc, ratio=0.9)
        ok = m >= 0
        correct = a.landmark[ok] == b.landmark[m[ok]]
        shared = np.isin(a.landmark[a.landmark >= 0], b.landmark).sum()
        assert correct.mean() >= 0.99 and ok.sum() >= 0.8 * shared, (i, j, correct.mean(), ok.sum(), shared)
