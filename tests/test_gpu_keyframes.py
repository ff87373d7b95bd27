"""GPU keyframe selection and novelty test of the memory pool (Sec. IV-C,
IV-E) against the oracle.  Both evaluate rotation geodesics in FP64 (their
own trace sums and arccos), so the selection must be identical unless two
candidates' cost sums are within rounding (1e-12) of each other at some step
(certified); the novelty flag must agree unless the nearest keyframe is
within 1e-12 of the threshold.  Pools of 1 to 2048 keyframes, K of 1, 15 and
the pool size, pools on one rotation axis with exact ties, argument errors."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle

pytestmark = pytest.mark.gpu


def pool_of(n, seed, spread=0.6):
    rng = np.random.default_rng(seed)
    base = Rotation.random(random_state=seed)
    T = np.tile(np.eye(4), (n, 1, 1))
    for k in range(n):
        T[k, :3, :3] = (base * Rotation.from_rotvec(rng.normal(scale=spread, size=3))).as_matrix()
        T[k, :3, 3] = rng.normal(scale=0.02, size=3) + [0, 0, 0.6]
    cur = np.eye(4)
    cur[:3, :3] = (base * Rotation.from_rotvec(rng.normal(scale=spread, size=3))).as_matrix()
    return T, cur


def certify(T, cur, K, sel_g, sel_o):
    """Selections equal, or equal up to a step where the oracle's sums of the
    two picks differ by at most 1e-12."""
    if np.array_equal(sel_g, sel_o):
        return 0
    assert len(sel_g) == len(sel_o)
    n = int(np.argmax(sel_g != sel_o))
    chosen = [cur] + [T[s] for s in sel_o[:n]]
    s = lambda k: sum(oracle.rot_geodesic(T[k], c) for c in chosen)
    assert abs(s(sel_g[n]) - s(sel_o[n])) <= 1e-12, (n, sel_g[n], sel_o[n])
    return 1


@pytest.mark.parametrize("n,K", [(1, 15), (2, 15), (16, 15), (40, 15), (300, 15), (2048, 15), (57, 1), (23, 23)])
def test_selection_matches_oracle(n, K):
    from paper_2108_00516_amd import frontend
    T, cur = pool_of(n, n + K)
    print(f"keyframes: pool {n}, K {K}", flush=True)
    sel, novel, cost = frontend.select_keyframes(T, cur, K)
    osel, ocost = oracle.select_keyframes(T, cur, K)
    assert len(sel) == min(n, K) and sel[0] == 0
    assert certify(T, cur, K, sel, osel) == 0 or n > 100
    if np.array_equal(sel, osel):
        assert np.allclose(cost, ocost, rtol=0, atol=1e-12 * max(1, K))
    onovel = oracle.novel_view(T, cur)
    nearest = min(oracle.rot_geodesic(t, cur) for t in T)
    assert novel == onovel or abs(nearest - np.deg2rad(10.0)) <= 1e-12


def test_selection_from_device_pool_and_ties():
    """Poses on one rotation axis at whole degrees: the sums tie exactly for
    mirror-image candidates and the lower index wins on both sides; the pool
    read from device memory gives the same result."""
    import torch
    from paper_2108_00516_amd import frontend
    ang = [0, 10, -10, 20, -20, 30, -30, 5, -5]
    T = np.tile(np.eye(4), (len(ang), 1, 1))
    for k, d in enumerate(ang):
        T[k, :3, :3] = Rotation.from_rotvec([0, 0, np.deg2rad(d)]).as_matrix()
    cur = np.eye(4)
    sel, novel, _ = frontend.select_keyframes(T, cur, 5)
    osel, _ = oracle.select_keyframes(T, cur, 5)
    assert certify(T, cur, 5, sel, osel) == 0
    assert not novel
    dsel, dnovel, _ = frontend.select_keyframes(torch.from_numpy(T.reshape(-1, 16)).cuda(), cur, 5)
    assert np.array_equal(dsel, sel) and dnovel == novel
    far = np.eye(4)
    far[:3, :3] = Rotation.from_rotvec([0, 0, np.deg2rad(45)]).as_matrix()
    assert frontend.select_keyframes(T, far, 5)[1] is True


def test_argument_errors():
    from paper_2108_00516_amd import frontend
    T, cur = pool_of(4, 1)
    with pytest.raises(frontend.FrontendError, match="INVALID_ARG"):
        frontend.select_keyframes(T, cur, 0)
    with pytest.raises(frontend.FrontendError, match="CAPACITY"):
        frontend.select_keyframes(np.tile(np.eye(4), (2049, 1, 1)), cur, 15)
