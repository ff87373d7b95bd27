"""GPU: learned correspondence weighting — the trainer kernels (forward,
loss/gradient, Adam) against the FP64 oracle, the association features and
network weights, the pruning pass, and whole learned optimisations against the
oracle; then the gain of a trained network on windows whose masks leak onto
the background.

The network runs "in FP16" on both sides: binary16 parameters, every layer's
input (features, both hidden layers' activations) rounded to binary16; the GPU
sums in FP32, the oracle exactly.  Each network output is checked against a
bound derived per sample from that rule (a rounding-boundary flip is allowed
only where the FP32 sums or the feature differences reach a binary16
boundary).  Pruning decisions are integers decided in floating point: the
GPU's kept pixels are compared with the oracle's own selection, and every
differing pixel is certified to lie at the threshold within the score bound;
the end-to-end comparison then gives the oracle the certified GPU set."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import certify_pruning, max_pose_diff, net_sigma_bound

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
        # every output within its derived bound, on the GPU's own features and
        # on the oracle's (whose binary16 inputs may differ from the GPU's)
        net = p16.astype(np.float64)
        b, flips = net_sigma_bound(net, f[same], f[same])
        d = np.abs(sg[same] - oracle.mlp_forward_half(net, f[same].astype(np.float64)))
        say(f"  sigma on the GPU features: max {d.max():.2e}, max/bound {np.max(d / b):.3f}, "
            f"{int(flips.sum())} samples near a binary16 boundary")
        assert np.all(d <= b)
        b, flips = net_sigma_bound(net, f[same], fo[same])
        d = np.abs(sg[same] - oracle.mlp_forward_half(net, fo[same]))
        say(f"  sigma on the oracle features: max {d.max():.2e}, max/bound {np.max(d / b):.3f}, "
            f"{int(flips.sum())} samples with a possible flip")
        assert np.all(d <= b)
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


def certified_keep(g, pg, pb, p16, frac, label):
    """The GPU's pruning pass against the oracle's own at the starting poses:
    every network output of the iteration-0 association within its derived
    bound, every source score within the largest bound over its targets (where
    all target decisions agree), and every differing keep decision certified at
    the threshold (certify_pruning).  Returns the GPU's keep mask."""
    N, hw = g.n_frames, g.width * g.height
    net = p16.astype(np.float64)
    score_g, keep_g = pg.prune()
    check_selection(score_g, keep_g, frac)
    score_o = pb.prune_scores(g.poses_init).reshape(N, hw)
    keep_o = pb.prune_select(score_o.reshape(N, g.height, g.width), frac).reshape(N, hw)
    t_pix = np.zeros((N, hw))
    uncertain = np.zeros((N, hw), bool)
    n_flip = n_pp = 0
    for i in range(N):
        pairs = [(i, j) for j in range(N) if j != i]
        To, Fo = pb.pairs_features(g.poses_init, pairs, 0)
        for q, (_, j) in enumerate(pairs):
            fg, sg, tg = pg.pair_features(i, j, 0, sigma=True)
            to = To[q]
            uncertain[i] |= ((tg >= 0) != (to >= 0)) | ((tg >= 0) & (tg != to))
            both = (tg >= 0) & (tg == to)
            b, flips = net_sigma_bound(net, fg[both], Fo[q][both])
            d = np.abs(sg[both] - oracle.mlp_forward_half(net, Fo[q][both]))
            assert np.all(d <= b), f"pair ({i},{j}): network output off its bound"
            t_pix[i][both] = np.maximum(t_pix[i][both], b)
            n_flip += int(flips.sum())
            n_pp += int(both.sum())
    n_diff, n_cert = certify_pruning(score_g, keep_g, score_o, keep_o, t_pix, uncertain, frac)
    say(f"{label}: {n_pp} gated-in pixel-pairs ({n_flip} with a possible binary16 flip), "
        f"{int(uncertain.sum())} sources with a differing association; keep differs at {n_diff} of "
        f"{int((score_o >= 0).sum())} sources ({n_cert} certified at the threshold, the rest uncertain)")
    return keep_g


@pytest.mark.parametrize("frac", [0.25, 0.5])
def test_prune_scores_and_selection(frac):
    g = synth.make_graph("T")
    p16 = rand_params(5)
    pg = gpu_graph(g, learned_cfg(g, prune_frac=frac), p16)
    pb = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=p16.astype(np.float64)))
    keep = certified_keep(g, pg, pb, p16, frac, f"T frac {frac}")
    score, keep2 = pg.prune()
    assert np.array_equal(keep, keep2)
    # the oracle's own selection from the GPU scores is the GPU's selection
    ko = pb.prune_select(score.reshape(g.n_frames, g.height, g.width).astype(np.float64), frac)
    assert np.array_equal(ko.reshape(g.n_frames, -1).astype(bool), keep)
    pg.close()


@pytest.mark.parametrize("params", ["random", "flat"])
def test_prune_selection_beyond_staged_keys(params):
    """Source lists longer than the select holds in LDS (32,768 keys; 640x480
    with the masks grown by 40 pixels gives about 56k sources a frame) take the
    select that reads its keys from global memory: its keep mask is the
    definition's and the oracle's selection from the same scores, also when
    every gated-in score ties (flat parameters)."""
    g = synth.make_graph("T", n_frames=3, width=640, height=480, mask_dilate=40)
    if params == "random":
        p16 = rand_params(7)
    else:
        p16 = np.zeros(1313, np.float16)
        p16[1312] = 2.0
    pg = gpu_graph(g, learned_cfg(g, prune_frac=0.25), p16)
    score, keep = pg.prune()
    V = (score >= 0).sum(axis=1)
    say(f"sources per frame {V.tolist()}")
    assert V.max() > 32768
    check_selection(score, keep, 0.25)
    pb = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=p16.astype(np.float64)))
    ko = pb.prune_select(score.reshape(g.n_frames, g.height, g.width).astype(np.float64), 0.25)
    assert np.array_equal(ko.reshape(g.n_frames, -1).astype(bool), keep)
    pg.close()


def test_prune_threshold_inside_zero_scores():
    """A threshold inside the zero scores (sources gated in nowhere), the tie
    the select resolves from its first digit's count of exact zeros: the keep
    mask is the definition's (the lowest positions of the zeros dropped) and
    the oracle's selection from the same scores."""
    g = synth.make_graph("T", mask_dilate=8)
    p16 = rand_params(5)
    pg = gpu_graph(g, learned_cfg(g, prune_frac=0.25), p16)
    score, _ = pg.prune()
    pg.close()
    src = score >= 0
    V = src.sum(axis=1)
    zeros = (src & (score == 0)).sum(axis=1)
    say(f"sources {V.tolist()}, zero scores {zeros.tolist()}")
    assert zeros.min() >= 8
    frac = 0.5 * float((zeros / V).min())
    pg = gpu_graph(g, learned_cfg(g, prune_frac=frac), p16)
    score, keep = pg.prune()
    check_selection(score, keep, frac)
    # every dropped source is a zero score
    assert np.all(score[src & ~keep] == 0)
    pb = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=p16.astype(np.float64)))
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

def shipped_weights():
    import os
    from paper_2108_00516_amd import learn
    path = os.path.join(os.path.dirname(learn.__file__), "weights", "weightnet.npy")
    return np.load(path).astype(np.float16)


@pytest.mark.parametrize("name,frac,weights", [("T", 0.25, "rand"), ("T", 0.0, "rand"), ("P", 0.25, "rand"),
                                               ("P", 0.25, "shipped"), ("L", 0.25, "shipped")])
def test_learned_optimize_matches_oracle(name, frac, weights):
    """Seven learned iterations against the oracle: the pruning decisions are
    certified against the oracle's own (certified_keep) and the oracle is then
    given the GPU's kept pixels; each side takes its own association decisions
    in every iteration.  L is the learned-weighting workload: 20 keyframes at
    640x480, 25 % pruned, the shipped network."""
    g = synth.make_graph(name)
    p16 = rand_params(7) if weights == "rand" else shipped_weights()
    say(f"learned optimise {name} ({g.n_frames} keyframes), prune {frac}, {weights} weights")
    pg = gpu_graph(g, learned_cfg(g, prune_frac=frac), p16)
    P = oracle.Params(mlp=p16.astype(np.float64), mlp_iters=7)
    pb = oracle.OracleProblem.from_synth(g, P)
    keep = None
    if frac > 0:
        # the pass optimize runs at the same starting poses
        keep = certified_keep(g, pg, pb, p16, frac, name)
    st = pg.optimize()
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
    # a second optimisation from the same poses and a fresh graph reproduce
    # the result bit for bit
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
    P = oracle.Params(mlp=p16.astype(np.float64), mlp_iters=7)
    pb = oracle.OracleProblem.from_synth(g, P)
    keep = certified_keep(g, pg, pb, p16, 0.25, "T linearize")
    H, gv, st = pg.linearize()
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
