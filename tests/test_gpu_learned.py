"""GPU: learned correspondence weighting — the trainer kernels (forward,
loss/gradient, Adam) against the FP64 oracle, the association features and
network weights, the pruning pass, and whole learned optimisations against the
oracle taking the same pruning decisions; then the gain of a trained network
on windows whose masks leak onto the background.

Readings shared with the oracle: the network runs on the fp16 parameters
widened exactly to FP32 (GPU) / FP64 (oracle); float-decided integers (which
pixels are pruned) are compared on one decision set: the oracle is given the
GPU's kept pixels, and the GPU's choice is checked to be exactly the lowest
scores by (score, position) of its own scores, and its scores against the
oracle's."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import max_pose_diff

pytestmark = pytest.mark.gpu

LEARNED_POSE_TOL = 1e-5   # rad / m, learned optimisation vs oracle with the same kept pixels


@pytest.fixture(scope="module", autouse=True)
def cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda")
    oracle.build(force=False)
    oracle.set_threads(16)


def say(msg):
    print(msg, flush=True)


def rand_params(seed, scale=1.0, out_bias=0.5):
    """fp16 parameters whose network output spreads over (0.2, 0.9) on the
    feature ranges of the association."""
    from paper_2108_00516_amd.learn import init_params
    p = init_params(seed) * scale
    p[1312] = out_bias
    return p.astype(np.float16)


def features_like(rng, n):
    """Feature vectors in the ranges the association produces."""
    x = np.empty((n, 6), np.float32)
    x[:, 0] = rng.uniform(-2.0, 2.0, n)
    x[:, 1] = rng.uniform(0.0, 1.0, n)
    x[:, 2] = rng.uniform(0.4, 1.4, n)
    x[:, 3] = rng.uniform(0.0, 1.0, n)
    x[:, 4] = rng.uniform(0.0, 1.0, n)
    x[:, 5] = rng.integers(0, 7, n) / 6.0
    return x


def learned_cfg(g, **kw):
    from paper_2108_00516_amd import Config, _lib
    return Config(max_frames=max(g.n_frames, 2), weighting=_lib.PG_WEIGHT_LEARNED, **kw)


def gpu_graph(g, cfg, p16):
    from paper_2108_00516_amd import from_synth
    pg = from_synth(g, cfg, device_inputs=True)
    pg.set_mlp(p16)
    return pg


# ------------------------------------------------------------ trainer kernels

def test_forward_matches_oracle():
    import torch
    from paper_2108_00516_amd import MlpTrainer
    rng = np.random.default_rng(5)
    p = rand_params(1).astype(np.float32)
    x = features_like(rng, 10_001)
    tr = MlpTrainer(len(x))
    tr.set_params(p)
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(len(x), device="cuda")
    tr.forward(xd, y)
    ref = oracle.mlp_forward(p.astype(np.float64), x.astype(np.float64))
    err = np.abs(y.cpu().numpy() - ref).max()
    say(f"forward max |err| {err:.2e}")
    assert err <= 2e-6
    assert np.array_equal(tr.params(), p)
    assert np.array_equal(tr.params_fp16(), p.astype(np.float16))
    tr.close()


@pytest.mark.parametrize("n", [1, 63, 64, 10_001])
def test_loss_and_gradient_match_oracle(n):
    """Gradient check: the GPU's mean BCE and its 1313-entry gradient against
    the oracle's FP64 backpropagation (itself pinned against central
    differences on the CPU).  FP32 products and 64-sample FP32 block sums:
    every entry within 1e-4 of the largest of its layer plus 1e-6 relative."""
    import torch
    from paper_2108_00516_amd import MlpTrainer
    rng = np.random.default_rng(n)
    p = rand_params(2).astype(np.float32)
    x = features_like(rng, n)
    y = (rng.random(n) < 0.6).astype(np.float32)
    tr = MlpTrainer(max(n, 64))
    tr.set_params(p)
    loss, g = tr.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    lo, go = oracle.mlp_bce(p.astype(np.float64), x.astype(np.float64), y.astype(np.float64))
    say(f"n={n}: loss {loss:.6f} vs {lo:.6f}; max |dgrad| {np.abs(g - go).max():.2e} of {np.abs(go).max():.2e}")
    assert loss == pytest.approx(lo, rel=1e-5, abs=1e-7)
    for a, b in [(0, 192), (192, 224), (224, 1248), (1248, 1280), (1280, 1312), (1312, 1313)]:
        scale = np.abs(go[a:b]).max()
        assert np.all(np.abs(g[a:b] - go[a:b]) <= 1e-4 * scale + 1e-6 * np.abs(go[a:b]) + 1e-9), (a, b)
    tr.close()


def test_adam_step_matches_reference_and_training_descends():
    import torch
    from paper_2108_00516_amd import MlpTrainer
    rng = np.random.default_rng(9)
    n = 20_000
    x = features_like(rng, n)
    # a separable toy rule: small residual and near depth -> inlier
    y = ((np.abs(x[:, 0]) < 0.8) & (x[:, 2] < 1.0)).astype(np.float32)
    p = rand_params(3).astype(np.float32)
    tr = MlpTrainer(n)
    tr.set_params(p)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    lr = 1e-3
    l0 = tr.adam_step(xd, yd, lr, want_loss=True)
    # first bias-corrected Adam step: delta = -lr * g / (|g| + eps)
    _, go = oracle.mlp_bce(p.astype(np.float64), x.astype(np.float64), y.astype(np.float64))
    p1 = tr.params().astype(np.float64)
    big = np.abs(go) > 1e-4 * np.abs(go).max()
    expect = p.astype(np.float64) - lr * go / (np.abs(go) + 1e-8)
    assert np.abs(p1 - expect)[big].max() <= 1e-6
    assert np.all(np.abs(p1 - p)[~big] <= lr * (1 + 1e-6))
    losses = [l0]
    for s in range(300):
        losses.append(tr.adam_step(xd, yd, 3e-3, want_loss=(s % 100 == 99)) or losses[-1])
    lf, _ = tr.loss_grad(xd, yd)
    say(f"BCE {l0:.4f} -> {lf:.4f} after 301 Adam steps")
    assert lf < 0.5 * l0
    tr.close()


# ------------------------------------------------- association features / weights

def test_pair_features_and_weights_match_oracle():
    from paper_2108_00516_amd import Config, from_synth
    g = synth.make_graph("T")
    p16 = rand_params(4)
    pg = from_synth(g, Config(max_frames=4), device_inputs=True)
    pg.set_mlp(p16)
    P = oracle.Params(mlp=p16.astype(np.float64), mlp_iters=7)
    pb = oracle.OracleProblem.from_synth(g, P)
    for (i, j, it) in [(0, 1, 0), (2, 1, 3), (3, 0, 6)]:
        f, sg, t = pg.pair_features(i, j, it, sigma=True)
        to, fo = pb.pair_features(g.poses_init, i, j, it)
        same = (t == to) & (t >= 0)
        assert same.sum() > 0.97 * (to >= 0).sum()
        df = np.abs(f[same] - fo[same])
        say(f"pair ({i},{j}) it {it}: {same.sum()} pixels, max |df| per feature {df.max(axis=0)}")
        # r / huber and |s - p| / gate carry FP32 rounding of millimetre
        # differences; the others are O(1e-6)
        assert np.all(df.max(axis=0) <= np.array([2e-4, 2e-5, 1e-6, 1e-6, 2e-4, 0.0]))
        # the association evaluates the network with fp16 inputs and first
        # activations (matrix cores); the oracle rounds the same values.  On
        # the GPU's own features the outputs agree to FP32 summation error,
        # except where a first-layer activation sits on a binary16 rounding
        # boundary (one fp16 ulp moves sigma by < 1e-3); on the oracle's
        # features (within 2e-4 of the GPU's), an input itself may round to
        # the neighbouring binary16 value
        net = p16.astype(np.float64)
        d = np.abs(sg[same] - oracle.mlp_forward_half(net, f[same].astype(np.float64)))
        say(f"  sigma on the GPU features: {100 * np.mean(d <= 2e-6):.3f}% within 2e-6, max {d.max():.2e}")
        assert np.mean(d <= 2e-6) >= 0.999 and d.max() <= 2e-3
        d = np.abs(sg[same] - oracle.mlp_forward_half(net, fo[same]))
        say(f"  sigma on the oracle features: {100 * np.mean(d <= 2e-5):.3f}% within 2e-5, max {d.max():.2e}")
        assert np.mean(d <= 2e-5) >= 0.95 and d.max() <= 2e-3
        assert np.all(f[t < 0] == 0) and np.all(sg[t < 0] == 0)
    pg.close()


# ------------------------------------------------------------------ pruning

def check_selection(score, keep, frac):
    """keep must be exactly the complement of the floor(frac V) lowest
    (score, position) sources of each frame."""
    for f in range(score.shape[0]):
        src = np.flatnonzero(score[f] >= 0)
        V = len(src)
        drop = int(math.floor(frac * V))
        order = np.lexsort((src, score[f][src]))   # by score, then position
        want = np.zeros(score.shape[1], bool)
        want[src[order[drop:]]] = True
        assert np.array_equal(keep[f], want), f
        assert keep[f].sum() == V - drop


@pytest.mark.parametrize("frac", [0.25, 0.5])
def test_prune_scores_and_selection(frac):
    g = synth.make_graph("T")
    p16 = rand_params(5)
    pg = gpu_graph(g, learned_cfg(g, prune_frac=frac), p16)
    score, keep = pg.prune()
    check_selection(score, keep, frac)
    pb = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=p16.astype(np.float64)))
    so = pb.prune_scores(g.poses_init).reshape(g.n_frames, -1)
    assert np.array_equal(score < 0, so < 0)
    d = np.abs(score - so)[so >= 0]
    frac_close = np.mean(d <= 5e-5)
    say(f"frac {frac}: scores within 5e-5 for {100 * frac_close:.3f}% of sources (max {d.max():.2e})")
    # a source whose best target flips at a pixel-rounding tie may score differently
    assert frac_close >= 0.995
    # the oracle's own selection from the GPU scores is the GPU's selection
    ko = pb.prune_select(score.reshape(g.n_frames, g.height, g.width).astype(np.float64), frac)
    assert np.array_equal(ko.reshape(g.n_frames, -1).astype(bool), keep)
    pg.close()


def test_prune_edge_cases():
    from paper_2108_00516_amd import Config, PoseGraphError, from_synth
    g = synth.make_graph("T", n_frames=2)
    p16 = rand_params(6)
    # all scores tie (output bias dominates): the lowest positions are dropped
    flat = np.zeros(1313, np.float16)
    flat[1312] = 2.0
    pg = gpu_graph(g, learned_cfg(g, prune_frac=0.3), flat)
    score, keep = pg.prune()
    check_selection(score, keep, 0.3)
    pg.close()
    # frac 1: everything dropped; the dense term vanishes, the features remain
    pg = gpu_graph(g, learned_cfg(g, prune_frac=1.0), p16)
    score, keep = pg.prune()
    assert keep.sum() == 0
    st = pg.optimize(check=False)
    assert np.all(st["n_valid_g"] == 0)
    pg.close()
    # single frame
    g1 = synth.make_graph("T", n_frames=1)
    pg = gpu_graph(g1, learned_cfg(g1, prune_frac=0.25), p16)
    score, keep = pg.prune()
    check_selection(score, keep, 0.25)
    assert np.all(score[score >= 0] == 0)
    pg.close()
    # learned weighting without parameters, pruning without learned weighting
    pg = from_synth(g, learned_cfg(g), device_inputs=True)
    with pytest.raises(PoseGraphError):
        pg.optimize()
    pg.close()
    pg = from_synth(g, Config(max_frames=2), device_inputs=True)
    with pytest.raises(PoseGraphError):
        pg.prune()
    pg.close()


# ---------------------------------------------------------- learned optimise

@pytest.mark.parametrize("name,frac", [("T", 0.25), ("T", 0.0), ("P", 0.25)])
def test_learned_optimize_matches_oracle(name, frac):
    g = synth.make_graph(name)
    p16 = rand_params(7)
    say(f"learned optimise {name} ({g.n_frames} keyframes), prune {frac}")
    pg = gpu_graph(g, learned_cfg(g, prune_frac=frac), p16)
    keep = None
    if frac > 0:
        _, keep = pg.prune()          # the pass optimize runs at the same starting poses
    st = pg.optimize()
    P = oracle.Params(mlp=p16.astype(np.float64), mlp_iters=7)
    pb = oracle.OracleProblem.from_synth(g, P)
    if keep is not None:
        pb.set_keep(keep.reshape(g.n_frames, g.height, g.width))
    Po, so = pb.optimize(g.poses_init, 7)
    dr, dt = max_pose_diff(pg.poses, Po)
    say(f"  vs oracle {dr:.2e} rad {dt:.2e} m; energy_g {st['energy_g'][0]:.6e} vs {so['energy_g'][0]:.6e}")
    assert dr <= LEARNED_POSE_TOL and dt <= LEARNED_POSE_TOL
    assert st["energy_g"][0] == pytest.approx(so["energy_g"][0], rel=1e-4)
    if frac > 0:
        V = sum(int(pg.frame_info(f, with_map=False)[1]) for f in range(g.n_frames))
        assert st["src_pixels"] == (g.n_frames - 1) * int(keep.sum())
        assert int(keep.sum()) == V - sum(math.floor(frac * pg.frame_info(f, with_map=False)[1])
                                          for f in range(g.n_frames))
    # a graph replay reproduces the result bit for bit
    pg.set_poses(g.poses_init)
    P1 = pg.poses
    pg.optimize()
    pg2 = gpu_graph(g, learned_cfg(g, prune_frac=frac), p16)
    pg2.optimize()
    assert np.array_equal(pg.poses, pg2.poses)
    assert not np.array_equal(P1, pg.poses)
    pg.close()
    pg2.close()


def test_learned_linearize_matches_oracle():
    """Normal equations of the first learned iteration (pruned at the current
    poses) against the oracle's on the GPU's association and pruning
    decisions."""
    g = synth.make_graph("T")
    p16 = rand_params(8)
    pg = gpu_graph(g, learned_cfg(g, prune_frac=0.25), p16)
    _, keep = pg.prune()
    H, gv, st = pg.linearize()
    P = oracle.Params(mlp=p16.astype(np.float64), mlp_iters=7)
    pb = oracle.OracleProblem.from_synth(g, P)
    pb.set_keep(keep.reshape(g.n_frames, g.height, g.width))
    dec = np.stack([pg.associate(i, j)[0] for (i, j) in pb.ordered_pairs()])
    lin = pb.linearize_given(g.poses_init, dec)
    rel = np.linalg.norm(H - lin["H"]) / np.linalg.norm(lin["H"])
    say(f"learned H rel error {rel:.2e}")
    assert np.all(np.abs(H - lin["H"]) <= 1e-5 * lin["H_abs"] + 1e-6 * np.abs(lin["H"]).max())
    assert np.all(np.abs(gv - lin["g"]) <= 1e-5 * lin["g_abs"] + 1e-6 * lin["g_abs"].max())
    assert st["n_valid_g"] == lin["n_valid_g"]
    pg.close()


# -------------------------------------------------------------------- gain

def test_trained_network_reduces_error_of_leaky_masks():
    """Train on windows whose masks leak 4 px onto the back wall (labels from
    the plain optimiser on the true masks), then compare on held-out leaky
    windows: the learned optimiser with 25% of the pixels pruned must end
    closer to the ground truth than the plain one."""
    from paper_2108_00516_amd import Config, from_synth, learn
    train_seeds, test_seeds = [20, 21, 22, 23, 24, 25], [30, 31, 32, 33]
    windows = []
    for s in train_seeds:
        clean = synth.make_graph("T", seed=s)
        leaky = synth.make_graph("T", seed=s, mask_dilate=4)
        windows.append((leaky, learn.reference_poses(clean)))
    x, y = learn.collect(windows)
    say(f"{x.shape[0]} samples, {float(y.mean()):.3f} labelled inlier")
    p16, tr = learn.train(x, y, steps=300, log=say)
    tr.close()
    errs = {"plain": [], "learned": []}
    for s in test_seeds:
        g = synth.make_graph("T", seed=s, mask_dilate=4)
        for kind in errs:
            if kind == "plain":
                pg = from_synth(g, Config(max_frames=4), device_inputs=True)
            else:
                pg = gpu_graph(g, learned_cfg(g, prune_frac=0.25), p16)
            pg.optimize(check=False)
            e = max(oracle.pose_error(pg.poses[k], g.poses_gt[k])[0] for k in range(g.n_frames))
            errs[kind].append(e)
            pg.close()
    say("max rotation error vs ground truth, plain: " + ", ".join(f"{e:.2e}" for e in errs["plain"]))
    say("                                 learned: " + ", ".join(f"{e:.2e}" for e in errs["learned"]))
    assert np.mean(errs["learned"]) < np.mean(errs["plain"])
