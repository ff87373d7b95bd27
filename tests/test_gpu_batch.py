"""GPU: many independent windows of uneven node counts and resolutions in one
batched schedule (one launch per phase for all graphs, replayed as a hipGraph).
Each graph's result must equal its own single-graph run bit for bit, and the
oracle's within the pose tolerance."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import POSE_TOL_M, POSE_TOL_RAD, max_pose_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda")
    oracle.build(force=False)
    oracle.set_threads(16)


def gpu_graph(g, **cfg):
    from paper_2108_00516_amd import Config, from_synth
    return from_synth(g, Config(max_frames=max(g.n_frames, 2), **cfg), device_inputs=True)


def say(msg):
    print(msg, flush=True)


def small_uneven():
    return [synth.make_graph("T", seed=3, n_frames=3),
            synth.make_graph("T", seed=4, n_frames=5, width=120, height=90),
            synth.make_graph("T", seed=5, n_frames=4, width=80, height=60),
            synth.make_graph("T", seed=6, n_frames=2)]


def test_small_batch_matches_oracle_and_single_runs():
    from paper_2108_00516_amd import optimize_batch
    graphs = small_uneven()
    say("batch of 4 uneven small windows")
    single = []
    for g in graphs:
        pg = gpu_graph(g)
        pg.optimize()
        single.append(pg.poses)
        pg.close()
    pgs = [gpu_graph(g) for g in graphs]
    rc, stats = optimize_batch(pgs)
    assert rc == 0
    for k, (g, pg) in enumerate(zip(graphs, pgs)):
        P = pg.poses
        assert np.array_equal(P, single[k]), k
        Po, so = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
        dr, dt = max_pose_diff(P, Po)
        say(f"  graph {k} ({g.n_frames} keyframes {g.width}x{g.height}): {dr:.2e} rad {dt:.2e} m")
        assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
        assert stats[k]["iters_done"] == 7
        assert np.array_equal(stats[k]["n_valid_f"], so["n_valid_f"])
    # replay the captured batch after resetting the poses
    for pg, g in zip(pgs, graphs):
        pg.set_poses(g.poses_init)
    rc, _ = optimize_batch(pgs)
    assert rc == 0
    for k, pg in enumerate(pgs):
        assert np.array_equal(pg.poses, single[k])
    for pg in pgs:
        pg.close()


def test_paper_sized_uneven_batch_equals_single_runs():
    from paper_2108_00516_amd import optimize_batch
    graphs = [synth.make_graph(f"B{k}") for k in (0, 4, 7, 2)]
    say("batch of 4 windows: " + ", ".join(f"{g.n_frames}@{g.width}x{g.height}" for g in graphs))
    single = []
    for g in graphs:
        pg = gpu_graph(g)
        pg.optimize()
        single.append(pg.poses)
        pg.close()
    pgs = [gpu_graph(g) for g in graphs]
    rc, stats = optimize_batch(pgs)
    assert rc == 0
    for k, pg in enumerate(pgs):
        assert np.array_equal(pg.poses, single[k]), k
    # the smallest one against the oracle as well
    g = graphs[1]
    Po, _ = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
    dr, dt = max_pose_diff(pgs[1].poses, Po)
    assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
    for pg in pgs:
        pg.close()


def test_batch_with_singular_member():
    from paper_2108_00516_amd import _lib, optimize_batch
    graphs = small_uneven()
    g = graphs[1]
    mask = g.mask.copy()
    mask[2] = 0
    graphs[1] = synth.SynthGraph(**{**g.__dict__, "mask": mask,
                                    "matches": [m for m in g.matches if 2 not in (m.i, m.j)]})
    say("batch with a singular member")
    pgs = [gpu_graph(x) for x in graphs]
    rc, stats = optimize_batch(pgs, check=False)
    assert rc == _lib.PG_ERR_SINGULAR
    assert stats[1]["iters_done"] == 0 and np.array_equal(pgs[1].poses, graphs[1].poses_init)
    for k in (0, 2, 3):
        assert stats[k]["iters_done"] == 7
        Po, _ = oracle.OracleProblem.from_synth(graphs[k]).optimize(graphs[k].poses_init, 7)
        dr, dt = max_pose_diff(pgs[k].poses, Po)
        assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
    for pg in pgs:
        pg.close()


def test_batch_rebuilds_after_a_change():
    from paper_2108_00516_amd import optimize_batch
    graphs = small_uneven()
    say("batch rebuilt after a match change")
    pgs = [gpu_graph(g) for g in graphs]
    optimize_batch(pgs)
    m = graphs[0].matches[0]
    half = len(m.uv_i) // 2
    pgs[0].add_matches(m.i, m.j, m.uv_i[:half], m.uv_j[:half])
    for pg, g in zip(pgs, graphs):
        pg.set_poses(g.poses_init)
    optimize_batch(pgs)
    ref = gpu_graph(graphs[0])
    ref.add_matches(m.i, m.j, m.uv_i[:half], m.uv_j[:half])
    ref.optimize()
    assert np.array_equal(pgs[0].poses, ref.poses)
    ref.close()
    for pg in pgs:
        pg.close()
