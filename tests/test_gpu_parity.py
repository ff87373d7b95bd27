"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Sizes span several association tiles with ragged tails
(tiny window: ~1.4k valid pixels per frame, 1024-pixel tiles; paper-scale
window: ~22k per frame), plus the full 640x480 10- and 20-keyframe windows."""
import functools
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import (G_REL_TOL, H_REL_TOL, POSE_TOL_M, POSE_TOL_RAD, certify_association,
                         check_normal_equations, gpu_decisions, max_pose_diff, near_half_integer, oracle_step)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda")
    oracle.build(force=False)
    oracle.set_threads(16)
    return torch


@functools.lru_cache(maxsize=None)
def graph(name, **kw):
    return synth.make_graph(name, **kw)


def gpu_graph(g, **cfg):
    from paper_2108_00516_amd import Config, from_synth
    c = Config(max_frames=max(g.n_frames, 2), **cfg)
    return from_synth(g, c, device_inputs=True)


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("name", ["T", "P"])
def test_preprocess_parity(name):
    g = graph(name)
    say(f"preprocess parity {name}")
    pg = gpu_graph(g)
    pb = oracle.OracleProblem.from_synth(g)
    for f in range(g.n_frames):
        m, nv = pg.frame_info(f)
        V, Nn, code = pb.preprocess(f)
        valid_o = code == 3
        valid_g = m[..., 3] > 0
        assert np.array_equal(valid_o, valid_g)
        assert nv == valid_o.sum()
        assert np.array_equal(m[..., 3][valid_g], g.depth[f][valid_g])
        assert np.abs(m[..., :3][valid_g] - Nn[valid_g]).max() < 1e-5
    pg.close()


def certify_assoc(name, g, pg, pb, pairs):
    return certify_association(name, pg, pb, pairs, g.poses_init)


@pytest.mark.parametrize("name,pairs", [("T", [(0, 1), (1, 0), (3, 1)]), ("P", [(0, 1), (3, 7), (9, 2)])])
def test_association_parity(name, pairs):
    g = graph(name)
    say(f"association parity {name} {pairs}")
    pg = gpu_graph(g)
    pb = oracle.OracleProblem.from_synth(g)
    nd = certify_assoc(name, g, pg, pb, pairs)
    say(f"  certified near-tie differences: {nd}")
    pg.close()



@pytest.mark.parametrize("name", ["T", "P"])
def test_linearize_parity(name):
    """Normal equations at the initial poses.  The association decisions are
    integers decided in floating point: every GPU/oracle difference must be a
    near-tie (certified pair by pair), and on the GPU's decision set the
    oracle's FP64 H, g and energies must match."""
    g = graph(name)
    say(f"linearize parity {name}")
    pg = gpu_graph(g)
    pb = oracle.OracleProblem.from_synth(g)
    nd = certify_assoc(name, g, pg, pb, pb.ordered_pairs())
    H, gv, st = pg.linearize()
    lin = pb.linearize_given(g.poses_init, gpu_decisions(pg, pb))
    rel = check_normal_equations(H, gv, lin)
    say(f"  decision near-ties {nd}; H rel Frobenius error {rel:.2e}")
    assert np.array_equal(H, H.T)
    assert st["n_valid_f"] == lin["n_valid_f"]
    assert st["n_valid_g"] == lin["n_valid_g"]
    assert st["energy_f"] == pytest.approx(lin["energy_f"], rel=1e-5)
    assert st["energy_g"] == pytest.approx(lin["energy_g"], rel=1e-5)
    pg.close()



@pytest.mark.parametrize("name,lf,lg,iters", [("T", 1.0, 1.0, 7), ("T", 0.5, 2.0, 7), ("T", 1.0, 0.0, 4),
                                              ("T", 0.0, 1.0, 4), ("P", 1.0, 1.0, 3)])
def test_per_iteration_parity(name, lf, lg, iters):
    """Every Gauss-Newton iteration on the same decision set: the GPU's normal
    equations against the oracle's on the GPU's decisions (1e-5), and the GPU's
    update against the oracle's step from those equations."""
    g = graph(name)
    say(f"per-iteration parity {name} lambda_f={lf} lambda_g={lg}")
    pg = gpu_graph(g, lambda_f=lf, lambda_g=lg, gn_iters=1)
    pb = oracle.OracleProblem.from_synth(g, oracle.Params(lambda_f=lf, lambda_g=lg))
    P = pg.poses
    for it in range(iters):
        dec = gpu_decisions(pg, pb)
        lin = pb.linearize_given(P, dec)
        H, gv, st = pg.linearize()
        rel = check_normal_equations(H, gv, lin)
        Q = oracle_step(lin, P, g.fixed)
        pg.optimize()
        P = pg.poses
        dr, dt = max_pose_diff(P, Q)
        say(f"  iteration {it}: H rel {rel:.2e}, step difference {dr:.2e} rad {dt:.2e} m")
        assert dr <= 1e-6 and dt <= 1e-6
    pg.close()


@pytest.mark.parametrize("name", ["T", "P", "X"])
def test_optimize_parity(name):
    g = graph(name)
    say(f"optimize parity {name} ({g.n_frames} keyframes {g.width}x{g.height}, 7 iterations)")
    pg = gpu_graph(g)
    st = pg.optimize()
    Pg = pg.poses
    Po, so = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
    dr, dt = max_pose_diff(Pg, Po)
    say(f"  max pose difference vs oracle: {dr:.2e} rad, {dt:.2e} m")
    assert st["iters_done"] == 7 and so["iters_done"] == 7
    assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
    assert np.allclose(st["energy_f"], so["energy_f"], rtol=1e-4)
    assert np.allclose(st["energy_g"], so["energy_g"], rtol=1e-3)
    assert np.array_equal(st["n_valid_f"], so["n_valid_f"])
    pg.close()


@pytest.mark.parametrize("name,fixed,solver", [("T", (0, 2), "GAUSS_JORDAN"), ("P", (0, 4, 7), "GAUSS_JORDAN"),
                                                ("P", (0, 4, 7), "CHOLESKY"), ("T", (0, 2), "LDL"),
                                                ("P", (0, 4, 7), "LDL"), ("P", (0, 4, 7), "PCG_MATRIX_FREE")])
def test_interior_fixed_nodes(name, fixed, solver):
    """Fixed nodes inside the window: the free-node system skips their rows and
    columns (node -> free position table), the poses of fixed nodes stay put."""
    from paper_2108_00516_amd import _lib
    g0 = graph(name)
    fx = np.zeros(g0.n_frames, np.int32)
    fx[list(fixed)] = 1
    g = synth.SynthGraph(**{**g0.__dict__, "fixed": fx})
    say(f"interior fixed nodes {fixed} {name}, {solver}")
    pg = gpu_graph(g, solver=getattr(_lib, "PG_SOLVER_" + solver))
    st = pg.optimize()
    Pg = pg.poses
    Po, so = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
    dr, dt = max_pose_diff(Pg, Po)
    say(f"  max pose difference vs oracle: {dr:.2e} rad, {dt:.2e} m")
    assert st["iters_done"] == 7 and so["iters_done"] == 7
    assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
    for k in fixed:
        assert np.array_equal(Pg[k], g.poses_init[k])
    pg.close()


def test_determinism_and_graph_replay():
    g = graph("T")
    say("determinism / graph replay T")
    import torch
    pg_plain = gpu_graph(g, use_graph=0)
    pg_graph = gpu_graph(g, use_graph=1)
    pg_plain.optimize()
    ref = pg_plain.poses
    for rep in range(4):
        pg_graph.set_poses(g.poses_init)
        pg_graph.optimize()
        assert np.array_equal(pg_graph.poses, ref), f"replay {rep}"
        # eager work of the program between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        torch.cuda.synchronize()
    pg_plain.set_poses(g.poses_init)
    pg_plain.optimize()
    assert np.array_equal(pg_plain.poses, ref)
    pg_plain.close()
    pg_graph.close()


@pytest.mark.parametrize("tile", [256, 512, 2048])
def test_tile_sizes(tile):
    g = graph("T")
    say(f"tile {tile} T")
    pg = gpu_graph(g, tile_pixels=tile)
    pg.optimize()
    Po, _ = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
    dr, dt = max_pose_diff(pg.poses, Po)
    assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
    pg.close()


@pytest.mark.parametrize("solver", ["PCG", "CHOLESKY", "GAUSS_JORDAN", "LDL", "PCG_MATRIX_FREE"])
def test_solvers_match(solver):
    from paper_2108_00516_amd import _lib
    g = graph("T")
    say(f"{solver} solver T")
    pg = gpu_graph(g, solver=getattr(_lib, "PG_SOLVER_" + solver))
    pg.optimize()
    Po, _ = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
    dr, dt = max_pose_diff(pg.poses, Po)
    assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
    pg.close()


def test_singular_window_keeps_poses():
    from paper_2108_00516_amd import PoseGraphError, _lib
    g0 = graph("T")
    say("singular window T")
    mask = g0.mask.copy()
    mask[2] = 0
    g = synth.SynthGraph(**{**g0.__dict__, "mask": mask,
                            "matches": [m for m in g0.matches if 2 not in (m.i, m.j)]})
    pg = gpu_graph(g)
    st = pg.optimize(check=False)
    assert st["status"] == _lib.PG_ERR_SINGULAR
    assert st["iters_done"] == 0
    assert np.array_equal(pg.poses, g.poses_init)
    Po, so = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
    assert so["status"] == oracle.ERR_SINGULAR and so["iters_done"] == 0
    with pytest.raises(PoseGraphError):
        pg.optimize()
    pg.close()


def test_all_fixed_and_single_frame():
    from paper_2108_00516_amd import Camera, Config, PoseGraph
    g = graph("T")
    say("all fixed / single frame T")
    pg = PoseGraph(Camera(g.width, g.height, g.fx, g.fy, g.cx, g.cy), Config(max_frames=4))
    for k in range(g.n_frames):
        pg.add_frame(g.depth[k], g.mask[k], g.poses_init[k], fixed=True)
    st = pg.optimize()
    assert st["iters_done"] == 7 and np.array_equal(pg.poses, g.poses_init)
    pg.close()
    pg = PoseGraph(Camera(g.width, g.height, g.fx, g.fy, g.cx, g.cy), Config(max_frames=4))
    pg.add_frame(g.depth[0], g.mask[0], g.poses_init[0], fixed=True)
    st = pg.optimize()
    assert st["iters_done"] == 7 and np.array_equal(pg.poses[0], g.poses_init[0])
    pg.close()


def test_host_and_device_inputs_agree():
    from paper_2108_00516_amd import Config, from_synth
    g = graph("T")
    say("host vs device inputs T")
    a = from_synth(g, Config(max_frames=4), device_inputs=False)
    b = from_synth(g, Config(max_frames=4), device_inputs=True)
    a.optimize()
    b.optimize()
    assert np.array_equal(a.poses, b.poses)
    a.close()
    b.close()


def test_nonfinite_depth_is_invalid():
    g0 = graph("T")
    say("non-finite depth T")
    depth = g0.depth.copy()
    rng = np.random.default_rng(9)
    for f in range(g0.n_frames):
        vv, uu = np.nonzero(g0.mask[f])
        sel = rng.choice(len(vv), 40, replace=False)
        depth[f, vv[sel[:20]], uu[sel[:20]]] = np.nan
        depth[f, vv[sel[20:30]], uu[sel[20:30]]] = np.inf
        depth[f, vv[sel[30:]], uu[sel[30:]]] = -1.0
    g = synth.SynthGraph(**{**g0.__dict__, "depth": depth})
    pg = gpu_graph(g)
    pg.optimize()
    Po, _ = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
    dr, dt = max_pose_diff(pg.poses, Po)
    assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
    pg.close()


def test_matches_replace_and_remove():
    g = graph("T")
    say("match replacement T")
    pg = gpu_graph(g)
    m0 = g.matches[0]
    # replace the first set by its first half, given in swapped order
    half = len(m0.uv_i) // 2
    pg.add_matches(m0.j, m0.i, m0.uv_j[:half], m0.uv_i[:half])
    # remove the last set
    ml = g.matches[-1]
    pg.add_matches(ml.i, ml.j, np.zeros((0, 2), np.float32), np.zeros((0, 2), np.float32))
    pg.optimize()
    matches = [synth.MatchSet(m0.i, m0.j, m0.uv_i[:half], m0.uv_j[:half], m0.inlier[:half])] + \
        list(g.matches[1:-1])
    pb = oracle.OracleProblem(g.depth, g.mask, g.fx, g.fy, g.cx, g.cy, g.fixed, matches)
    Po, so = pb.optimize(g.poses_init, 7)
    dr, dt = max_pose_diff(pg.poses, Po)
    assert dr <= POSE_TOL_RAD and dt <= POSE_TOL_M
    pg.close()


def test_abi_errors_on_gpu():
    from paper_2108_00516_amd import Camera, Config, PoseGraph, PoseGraphError, _lib
    g = graph("T")
    say("ABI errors")
    pg = PoseGraph(Camera(g.width, g.height, g.fx, g.fy, g.cx, g.cy), Config(max_frames=2))
    pg.add_frame(g.depth[0], g.mask[0], g.poses_init[0], fixed=True)
    bad = g.poses_init[1].copy()
    bad[0, 0] += 0.1
    with pytest.raises(PoseGraphError) as e:
        pg.add_frame(g.depth[1], g.mask[1], bad)
    assert e.value.status == _lib.PG_ERR_INVALID_ARG
    pg.add_frame(g.depth[1], g.mask[1], g.poses_init[1])
    with pytest.raises(PoseGraphError) as e:
        pg.add_frame(g.depth[2], g.mask[2], g.poses_init[2])
    assert e.value.status == _lib.PG_ERR_CAPACITY
    with pytest.raises(PoseGraphError) as e:
        pg.add_matches(0, 0, g.matches[0].uv_i, g.matches[0].uv_j)
    assert e.value.status == _lib.PG_ERR_INVALID_ARG
    with pytest.raises(PoseGraphError) as e:
        pg.get_pose(5)
    assert e.value.status == _lib.PG_ERR_INVALID_ARG
    with pytest.raises(PoseGraphError) as e:
        pg.set_mlp(np.zeros(10, np.float16))
    assert e.value.status == _lib.PG_ERR_INVALID_ARG
    pg.close()
    pg.close()  # destroy is NULL-safe / idempotent in the binding


def test_window_without_fixed_node_beyond_lds_is_refused():
    """32 frames with none fixed: 192 unknowns, whose packed solve layout
    exceeds the workgroup's LDS; the optimisation is refused with a capacity
    status before any launch and the poses are left as they were."""
    from paper_2108_00516_amd import Camera, Config, PoseGraph, PoseGraphError, _lib
    g = graph("T")
    say("32 free frames: LDS capacity")
    pg = PoseGraph(Camera(g.width, g.height, g.fx, g.fy, g.cx, g.cy), Config(max_frames=32))
    for k in range(32):
        pg.add_frame(g.depth[k % g.n_frames], g.mask[k % g.n_frames], g.poses_init[k % g.n_frames])
    with pytest.raises(PoseGraphError) as e:
        pg.optimize()
    assert e.value.status == _lib.PG_ERR_CAPACITY
    assert np.array_equal(pg.poses[:g.n_frames], g.poses_init)
    pg.close()


@pytest.mark.parametrize("use_graph", [0, 1])
def test_zero_iterations_and_continuation(use_graph):
    """Zero iterations return the start poses (no solve runs, the result block
    is copied back); a second optimize without set_poses starts from the
    first one's result (the start kernel reads the host mirror of the device
    poses): its first record is the energy at those poses, not at the start."""
    g = graph("T")
    say(f"zero iterations and continuation T, use_graph={use_graph}")
    pg0 = gpu_graph(g, gn_iters=0, use_graph=use_graph)
    st0 = pg0.optimize()
    assert st0["iters_done"] == 0
    assert np.array_equal(pg0.poses, g.poses_init)
    pg0.close()
    pg = gpu_graph(g, gn_iters=3, use_graph=use_graph)
    st1 = pg.optimize()
    P1 = pg.poses
    st2 = pg.optimize()
    assert st1["iters_done"] == 3 and st2["iters_done"] == 3
    ob = oracle.OracleProblem.from_synth(g)
    _, s_at_p1 = ob.optimize(P1, 1)
    say(f"  first energy: first optimize {st1['energy_g'][0]:.6e}, second {st2['energy_g'][0]:.6e}, "
        f"oracle at the first result {s_at_p1['energy_g'][0]:.6e}")
    assert np.isclose(st2["energy_g"][0], s_at_p1["energy_g"][0], rtol=1e-3)
    assert not np.isclose(st2["energy_g"][0], st1["energy_g"][0], rtol=1e-3)
    pg.close()


def test_matrix_free_pcg_against_explicit_normal_equations():
    """The matrix-free PCG (J^T W J applied from per-pair Gram blocks, never
    formed) against the direct solve of the explicitly assembled equations on
    the 10-keyframe window: the same association decisions and, with PCG
    converged to |r| <= 1e-12 |b|, the same steps (poses within 1e-9 after
    each of 7 iterations); the oracle within 1e-5 end to end; the PCG
    iteration counts reported; a capped PCG (3 iterations) reports 3 and ends
    elsewhere; a singular window fails as with the direct solve."""
    from paper_2108_00516_amd import _lib
    g = graph("P")
    say("matrix-free PCG vs explicit normal equations, P")
    mf = gpu_graph(g, solver=_lib.PG_SOLVER_PCG_MATRIX_FREE, gn_iters=1)
    dr_ = gpu_graph(g, solver=_lib.PG_SOLVER_LDL, gn_iters=1)
    for it in range(7):
        s1 = mf.optimize()
        dr_.optimize()
        a, b = mf.poses, dr_.poses
        d_r, d_t = max_pose_diff(a, b)
        say(f"  iteration {it}: PCG iterations {s1['pcg_iters'][0]}, difference {d_r:.2e} rad {d_t:.2e} m")
        assert 1 <= s1["pcg_iters"][0] < 500
        assert d_r <= 1e-9 and d_t <= 1e-9
        dr_.set_poses(a)          # continue both from the same poses
    mf.close()
    dr_.close()
    full = gpu_graph(g, solver=_lib.PG_SOLVER_PCG_MATRIX_FREE)
    st = full.optimize()
    Po, so = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
    d_r, d_t = max_pose_diff(full.poses, Po)
    say(f"  end to end vs oracle: {d_r:.2e} rad {d_t:.2e} m; PCG iterations {list(st['pcg_iters'])}")
    assert d_r <= POSE_TOL_RAD and d_t <= POSE_TOL_M
    assert np.array_equal(st["n_valid_f"], so["n_valid_f"])
    full.close()
    capped = gpu_graph(g, solver=_lib.PG_SOLVER_PCG_MATRIX_FREE, pcg_max_iters=3)
    st = capped.optimize()
    assert list(st["pcg_iters"]) == [3] * 7
    assert max_pose_diff(capped.poses, Po)[0] > 1e-7
    capped.close()
    mask = g.mask.copy()
    mask[2] = 0
    gs = synth.SynthGraph(**{**g.__dict__, "mask": mask,
                             "matches": [m for m in g.matches if 2 not in (m.i, m.j)]})
    sing = gpu_graph(gs, solver=_lib.PG_SOLVER_PCG_MATRIX_FREE)
    st = sing.optimize(check=False)
    assert st["status"] == _lib.PG_ERR_SINGULAR and st["iters_done"] == 0
    sing.close()
