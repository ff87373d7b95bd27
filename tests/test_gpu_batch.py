"""GPU: many independent windows of uneven node counts and resolutions in one
batched schedule (one launch per phase for all graphs; direct launches by
default, or the whole optimisation captured once and replayed as a hipGraph).
Each graph's result must equal its own single-graph run bit for bit, with
direct launches and with the graph replay alike, and the oracle's within the
pose tolerance: the 64 windows of the batched workload (seeds 100-163) each
against its single run and the oracle; small uneven batches with the learned
weighting and with the BF16x3 contraction against their single runs."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import POSE_TOL_M, POSE_TOL_RAD, max_pose_diff, per_iteration_certified

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
    # the same batch captured once and replayed as a hipGraph
    pgr = [gpu_graph(g, use_graph=1) for g in graphs]
    for rep in range(3):
        for pg, g in zip(pgr, graphs):
            pg.set_poses(g.poses_init)
        rc, _ = optimize_batch(pgr)
        assert rc == 0
        for k, pg in enumerate(pgr):
            assert np.array_equal(pg.poses, single[k]), (rep, k)
    for pg in pgr:
        pg.close()
    for k, (g, pg) in enumerate(zip(graphs, pgs)):
        P = pg.poses
        assert np.array_equal(P, single[k]), k
        Po, so = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
        dr, dt = max_pose_diff(P, Po)
        say(f"  graph {k} ({g.n_frames} keyframes {g.width}x{g.height}): {dr:.2e} rad {dt:.2e} m")
        assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
        assert stats[k]["iters_done"] == 7
        assert np.array_equal(stats[k]["n_valid_f"], so["n_valid_f"])
    # a second run of the same batch after resetting the poses
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


def _batch_graph(k):
    import synth as sy
    return sy.make_graph(f"B{k}")


def test_all_64_batched_windows_equal_single_runs_and_oracle():
    """The batched workload itself: 64 windows of 4-20 keyframes at 320x240,
    480x360 and 640x480 in one schedule; every window equal bit for bit to
    its single run.  Against the oracle, a window's 7 iterations end within
    1e-5 rad / m unless an association decision taken in FP32 on the GPU and
    in FP64 by the oracle (a projection within 1e-3 px of a pixel boundary,
    a gate within rounding) sends the two down slightly different paths:
    such windows (14 of the 64, up to 2e-5 rad) must stay within 1e-4 and
    pass the per-iteration check (every differing decision a certified
    near-tie, each step equal to the oracle's on the GPU's decisions within
    1e-6)."""
    import multiprocessing as mp
    from paper_2108_00516_amd import optimize_batch
    say("64-window batch: generating scenes")
    with mp.get_context("spawn").Pool(16) as pool:
        graphs = pool.map(_batch_graph, range(64))
    say("  " + " ".join(f"{g.n_frames}@{g.width}" for g in graphs))
    pgs = [gpu_graph(g) for g in graphs]
    rc, stats = optimize_batch(pgs)
    assert rc == 0
    batched = [pg.poses for pg in pgs]
    for pg in pgs:
        pg.close()
    worst, over = 0.0, []
    for k, g in enumerate(graphs):
        pg = gpu_graph(g)
        pg.optimize()
        assert np.array_equal(pg.poses, batched[k]), k
        pg.close()
        Po, so = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
        dr, dt = max_pose_diff(batched[k], Po)
        worst = max(worst, dr)
        assert np.array_equal(stats[k]["n_valid_f"], so["n_valid_f"]), k
        if not (dr <= POSE_TOL_RAD and dt <= POSE_TOL_M):
            over.append((k, dr, dt))
    say(f"  worst pose difference vs oracle over 64 windows: {worst:.2e} rad; beyond 1e-5: {over}")
    # windows whose end-to-end result passes the tolerance only through
    # association decisions that FP32 and FP64 take differently: each of their
    # iterations on the GPU's decisions matches the oracle's, and each
    # differing decision is a certified near-tie
    for k, dr, dt in over:
        assert dr <= 1e-4 and dt <= 1e-4, (k, dr, dt)
        n = per_iteration_certified(graphs[k])
        say(f"  window {k}: {dr:.2e} rad end to end; per iteration certified ({n} near-tie decisions)")
    assert len(over) <= 16


@pytest.mark.parametrize("form", ["learned", "bf16x3", "learned_bf16x3"])
def test_batched_forms_equal_single_runs(form):
    """The learned weighting (with pruning) and the BF16x3 contraction in a
    batched schedule: every window equal bit for bit to its single run."""
    from paper_2108_00516_amd import _lib, optimize_batch
    from paper_2108_00516_amd.learn import init_params
    kw = {}
    if "learned" in form:
        kw.update(weighting=_lib.PG_WEIGHT_LEARNED, prune_frac=0.25)
    if "bf16x3" in form:
        kw.update(precision=_lib.PG_PREC_BF16X3)
    p16 = init_params(3).astype(np.float16)
    graphs = small_uneven()
    say(f"batched {form}: 4 uneven windows")

    def make(g):
        pg = gpu_graph(g, **kw)
        if "learned" in form:
            pg.set_mlp(p16)
        return pg
    single = []
    for g in graphs:
        pg = make(g)
        pg.optimize()
        single.append(pg.poses)
        pg.close()
    pgs = [make(g) for g in graphs]
    rc, stats = optimize_batch(pgs)
    assert rc == 0
    for k, pg in enumerate(pgs):
        assert np.array_equal(pg.poses, single[k]), k
        assert stats[k]["iters_done"] == 7
        pg.close()
