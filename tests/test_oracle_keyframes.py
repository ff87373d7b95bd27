"""CPU pins of the oracle's keyframe memory pool (Sec. IV-C greedy selection
for the minimum H-subgraph over rotation geodesic distances; Sec. IV-E
novelty rule for admitting a frame): the geodesic against SciPy's rotation
angles, a hand-worked selection on one rotation axis, the cost bookkeeping
against direct sums, the greedy objective against exhaustive search over all
subsets of small pools (never below the optimum, equal to it on clustered
pools), pools no larger than K, and the 10-degree admission boundary."""
import itertools

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle


def pose(rot):
    T = np.eye(4)
    T[:3, :3] = rot.as_matrix() if hasattr(rot, "as_matrix") else rot
    T[:3, 3] = [0.01, -0.02, 0.6]
    return T


def angle(Ta, Tb):
    return Rotation.from_matrix(Ta[:3, :3].T @ Tb[:3, :3]).magnitude()


def test_geodesic_matches_scipy(oracle_lib):
    rs = Rotation.random(60, random_state=3)
    for k in range(0, 60, 2):
        a, b = pose(rs[k]), pose(rs[k + 1])
        assert oracle.rot_geodesic(a, b) == pytest.approx(angle(a, b), abs=1e-7)
        assert oracle.rot_geodesic(a, b) == oracle.rot_geodesic(b, a)
    a = pose(rs[0])
    assert oracle.rot_geodesic(a, a) == pytest.approx(0.0, abs=2e-8)
    flip = pose(rs[0] * Rotation.from_rotvec([0, np.pi, 0]))
    assert oracle.rot_geodesic(a, flip) == pytest.approx(np.pi, abs=1e-7)
    small = pose(rs[0] * Rotation.from_rotvec([0, 0, 0.05]))
    assert oracle.rot_geodesic(a, small) == pytest.approx(0.05, rel=1e-9)


def about_z(deg):
    return pose(Rotation.from_rotvec([0, 0, np.deg2rad(deg)]))


def test_hand_worked_selection(oracle_lib):
    """One axis, angles 0, 40, -3, 25, 14, 60 deg, current frame at 10 deg,
    K = 3: sums to {current, I_0} are 70, 16, 40, 18, 110 -> index 2; then
    adding |angle + 3|: 113, 68, 35, 173 -> index 4; the sums left after adding
    |angle - 14| are 139, 79, 219."""
    pool = np.stack([about_z(d) for d in (0, 40, -3, 25, 14, 60)])
    sel, cost = oracle.select_keyframes(pool, about_z(10), 3)
    assert list(sel) == [0, 2, 4]
    want = {1: 139, 3: 79, 5: 219}
    for k, v in want.items():
        assert np.rad2deg(cost[k]) == pytest.approx(v, abs=1e-6)


def test_cost_bookkeeping_and_order(oracle_lib):
    rng = np.random.default_rng(1)
    base = Rotation.random(random_state=5)
    pool = np.stack([pose(base * Rotation.from_rotvec(rng.normal(scale=0.4, size=3))) for _ in range(25)])
    cur = pose(base * Rotation.from_rotvec(rng.normal(scale=0.4, size=3)))
    sel, cost = oracle.select_keyframes(pool, cur, 9)
    assert sel[0] == 0 and len(set(sel)) == 9
    chosen = [cur] + [pool[s] for s in sel]
    for k in range(25):
        if k in sel:
            continue
        assert cost[k] == pytest.approx(sum(angle(pool[k], c) for c in chosen), abs=1e-9)
    # each added keyframe had the smallest sum at its turn
    for n in range(1, 9):
        picked = [cur] + [pool[s] for s in sel[:n]]
        sums = {k: sum(angle(pool[k], c) for c in picked) for k in range(25) if k not in sel[:n]}
        assert sums[sel[n]] <= min(sums.values()) + 1e-9


def objective(pool, cur, subset):
    members = [cur] + [pool[k] for k in subset]
    return sum(angle(a, b) for a, b in itertools.combinations(members, 2))


@pytest.mark.parametrize("clustered", [True, False])
def test_greedy_against_exhaustive_search(oracle_lib, clustered):
    """The minimum H-subgraph by brute force over every K-subset containing
    the initial frame: the greedy selection's objective is never below it,
    and on clustered pools (views near the current one plus far outliers) it
    is the optimum."""
    rng = np.random.default_rng(7 if clustered else 8)
    n, K = 9, 4
    for trial in range(6):
        base = Rotation.random(random_state=trial + (20 if clustered else 40))
        if clustered:
            near = [base * Rotation.from_rotvec(rng.normal(scale=0.05, size=3)) for _ in range(4)]
            far = [base * Rotation.from_rotvec(rng.normal(scale=1.2, size=3)) for _ in range(n - 4)]
            rots = [near[0]] + far[:2] + near[1:] + far[2:]
        else:
            rots = [base * Rotation.from_rotvec(rng.normal(scale=0.8, size=3)) for _ in range(n)]
        pool = np.stack([pose(r) for r in rots])
        cur = pose(base)
        sel, _ = oracle.select_keyframes(pool, cur, K)
        best = min(objective(pool, cur, (0,) + c) for c in itertools.combinations(range(1, n), K - 1))
        got = objective(pool, cur, sel)
        assert got >= best - 1e-9
        if clustered:
            assert got == pytest.approx(best, abs=1e-9)


def test_small_pools_select_everything(oracle_lib):
    pool = np.stack([about_z(d) for d in (0, 30, 15)])
    for K in (3, 5, 15):
        sel, _ = oracle.select_keyframes(pool, about_z(20), K)
        assert sel[0] == 0 and sorted(sel) == [0, 1, 2]
    sel, _ = oracle.select_keyframes(pool[:1], about_z(20), 15)
    assert list(sel) == [0]


def test_novelty_threshold(oracle_lib):
    pool = np.stack([about_z(d) for d in (0, 25, 50)])
    th = np.deg2rad(10.0)
    assert oracle.novel_view(pool, about_z(12.5 + 0.0), th) is True      # 12.5 from the nearest
    assert oracle.novel_view(pool, about_z(9.0), th) is False
    assert oracle.novel_view(pool, about_z(35.0001), th) is True
    assert oracle.novel_view(pool, about_z(34.999), th) is False
    assert oracle.novel_view(pool, about_z(-10.001), th) is True
    rng = np.random.default_rng(2)
    rp = [pose(Rotation.random(random_state=100 + k)) for k in range(30)]
    for k in range(20):
        cur = pose(Rotation.random(random_state=500 + k) if k % 2 else Rotation.from_matrix(rp[k][:3, :3]) *
                   Rotation.from_rotvec(rng.normal(scale=0.1, size=3)))
        want = min(angle(p, cur) for p in rp) > th
        assert oracle.novel_view(np.stack(rp), cur, th) == want
