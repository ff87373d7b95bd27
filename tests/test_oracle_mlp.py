"""Oracle pins of the learned weighting network: the gradient against central
finite differences of the loss, closed forms for zero weights, and the
layer structure checked by a hand-set network."""
import numpy as np
import pytest

import oracle


def random_params(rng, scale=0.3):
    return rng.normal(scale=scale, size=oracle.MLP_PARAMS)


def test_zero_weights_closed_form(oracle_lib):
    p = np.zeros(oracle.MLP_PARAMS)
    p[-1] = 0.7                       # b3
    x = np.random.default_rng(0).normal(size=(5, 6))
    y = oracle.mlp_forward(p, x)
    s = 1.0 / (1.0 + np.exp(-0.7))
    assert np.allclose(y, s, rtol=0, atol=1e-15)
    t = np.array([1, 0, 1, 1, 0], float)
    loss, g = oracle.mlp_bce(p, x, t)
    assert loss == pytest.approx(-(3 * np.log(s) + 2 * np.log(1 - s)) / 5, rel=1e-14)
    assert g[-1] == pytest.approx((5 * s - 3) / 5, rel=1e-14)
    assert np.all(g[:-1] == 0.0)


def test_hand_set_network():
    # W1 picks x0 into unit 0, W2 copies unit 0 into unit 0, W3 reads it:
    # y = sigmoid(2 relu(relu(x0)) - 1)
    p = np.zeros(oracle.MLP_PARAMS)
    p[0] = 1.0                        # W1[0, 0]
    W2 = 192 + 32
    p[W2 + 0] = 1.0                   # W2[0, 0]
    W3 = W2 + 1024 + 32
    p[W3 + 0] = 2.0
    p[W3 + 32] = -1.0                 # b3
    x = np.zeros((3, 6))
    x[:, 0] = [-1.0, 0.5, 2.0]
    y = oracle.mlp_forward(p, x)
    expect = 1.0 / (1.0 + np.exp(-(2.0 * np.maximum(x[:, 0], 0.0) - 1.0)))
    assert np.allclose(y, expect, rtol=0, atol=1e-15)


def test_gradient_finite_difference(oracle_lib):
    rng = np.random.default_rng(1)
    p = random_params(rng)
    x = rng.normal(size=(40, 6))
    t = (rng.random(40) < 0.5).astype(float)
    loss, g = oracle.mlp_bce(p, x, t)
    h = 1e-6
    idx = list(range(0, 192, 17)) + list(range(192, 224, 5)) + list(range(224, 1248, 97)) + \
        list(range(1248, 1280, 7)) + list(range(1280, 1313, 3))
    for k in idx:
        q = p.copy()
        q[k] += h
        lp, _ = oracle.mlp_bce(q, x, t, with_grad=False)
        q[k] -= 2 * h
        lm, _ = oracle.mlp_bce(q, x, t, with_grad=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-6 * abs(g[k]), k


def test_loss_is_stable_for_large_logits(oracle_lib):
    p = np.zeros(oracle.MLP_PARAMS)
    p[-1] = 800.0
    loss, _ = oracle.mlp_bce(p, np.zeros((2, 6)), np.array([1.0, 0.0]))
    assert np.isfinite(loss) and loss == pytest.approx(400.0, rel=1e-12)


# ---------------------------------------------------------------- learned GN

import synth  # noqa: E402


def const_net(value_logit):
    p = np.zeros(oracle.MLP_PARAMS)
    p[-1] = value_logit
    return p


def test_unit_network_reproduces_the_plain_method(oracle_lib):
    g = synth.make_graph("T")
    P0, s0 = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 4)
    pb = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=const_net(40.0)))   # sigmoid(40) == 1.0
    P1, s1 = pb.optimize(g.poses_init, 4)
    assert np.array_equal(P0, P1)
    assert np.array_equal(s0["energy_g"], s1["energy_g"])


def test_constant_network_scales_the_dense_term(oracle_lib):
    g = synth.make_graph("T")
    c = 0.3
    pb = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=const_net(np.log(c / (1 - c))), lambda_f=0.0))
    ref = oracle.OracleProblem.from_synth(g, oracle.Params(lambda_g=c, lambda_f=0.0))
    a, b = pb.linearize(g.poses_init), ref.linearize(g.poses_init)
    assert np.allclose(a["H"], b["H"], rtol=1e-13, atol=1e-13 * np.abs(b["H"]).max())
    assert np.allclose(a["g"], b["g"], rtol=1e-13, atol=1e-13 * np.abs(b["g"]).max())
    assert a["energy_g"] == pytest.approx(b["energy_g"], rel=1e-13)


def test_features_follow_their_definition(oracle_lib):
    g = synth.make_graph("T")
    pb = oracle.OracleProblem.from_synth(g)
    i, j, it = 1, 2, 3
    tgt, f = pb.pair_features(g.poses_init, i, j, iteration=it)
    t2, r, proj, gate = pb.associate(g.poses_init, i, j)
    assert np.array_equal(tgt, t2)
    V, _, _ = pb.preprocess(i)
    sel = np.flatnonzero(tgt >= 0)
    u, v = sel % g.width, sel // g.width
    expect = np.stack([r[sel] / 0.005,
                       np.degrees(np.arccos(np.clip(gate[sel, 1], -1, 1))) / 30.0,
                       V.reshape(-1, 3)[sel, 2] / 0.8,
                       np.hypot(u - g.cx, v - g.cy) / np.hypot(g.width / 2, g.height / 2),
                       gate[sel, 0] / 0.01,
                       np.full(len(sel), it / 6.0)], axis=1)
    assert np.allclose(f[sel], expect, rtol=1e-12, atol=1e-12)
    assert np.all(f[tgt < 0] == 0.0)


def test_pairs_features_equal_single_pair_calls(oracle_lib):
    g = synth.make_graph("T")
    pb = oracle.OracleProblem.from_synth(g)
    pairs = [(0, 1), (2, 1), (3, 0)]
    T, F = pb.pairs_features(g.poses_init, pairs, iteration=2)
    for q, (i, j) in enumerate(pairs):
        t, f = pb.pair_features(g.poses_init, i, j, iteration=2)
        assert np.array_equal(T[q], t) and np.array_equal(F[q], f)


def test_prune_scores_and_selection_brute_force(oracle_lib):
    g = synth.make_graph("T", width=80, height=60)
    rng = np.random.default_rng(4)
    net = rng.normal(scale=0.4, size=oracle.MLP_PARAMS)
    pb = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=net))
    sc = pb.prune_scores(g.poses_init)
    _, _, code = pb.preprocess(0)
    for i in range(g.n_frames):
        best = np.where(pb.preprocess(i)[2].ravel() == 3, 0.0, -1.0)
        for j in range(g.n_frames):
            if j == i:
                continue
            tgt, f = pb.pair_features(g.poses_init, i, j, iteration=0)
            sel = tgt >= 0
            y = np.zeros(len(tgt))
            y[sel] = oracle.mlp_forward_half(net, f[sel])
            best = np.where(sel, np.maximum(best, y), best)
        assert np.allclose(sc[i].ravel(), best, rtol=0, atol=1e-15)
    keep = pb.prune_select(sc, 0.25)
    for i in range(g.n_frames):
        s = sc[i].ravel()
        pos = np.flatnonzero(s >= 0)
        order = np.lexsort((pos, s[pos]))           # by score, then position
        drop = pos[order[:int(np.floor(0.25 * len(pos)))]]
        expect = np.zeros(s.size, np.uint8)
        expect[pos] = 1
        expect[drop] = 0
        assert np.array_equal(keep[i].ravel(), expect)


def test_pruned_optimize_equals_explicit_keep(oracle_lib):
    g = synth.make_graph("T")
    rng = np.random.default_rng(8)
    net = rng.normal(scale=0.4, size=oracle.MLP_PARAMS)
    a = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=net, prune_frac=0.25))
    Pa, sa = a.optimize(g.poses_init, 5)
    b = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=net))
    keep = b.prune_select(b.prune_scores(g.poses_init), 0.25)
    b.set_keep(keep)
    Pb, sb = b.optimize(g.poses_init, 5)
    assert np.array_equal(Pa, Pb)
    assert sa["n_valid_g"][0] < oracle.OracleProblem.from_synth(g).linearize(g.poses_init)["n_valid_g"]


def test_round_half_matches_numpy_binary16(oracle_lib):
    """Pinned to numpy's float64 -> float16 conversion (nearest, ties to even),
    over normal, subnormal, tie and overflow values."""
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.normal(scale=s, size=2000) for s in (1e-6, 1e-3, 1.0, 1e3, 3e4)])
    # exact ties between neighbouring binary16 values, and the extremes
    h = rng.normal(size=500).astype(np.float16).astype(np.float64)
    ties = h + np.spacing(h.astype(np.float16)).astype(np.float64) / 2
    xs = np.concatenate([xs, ties, [0.0, -0.0, 65504.0, 65519.0, 65520.0, -70000.0, 2.0 ** -24, 2.0 ** -25,
                                    3 * 2.0 ** -26, 6.0e-8]])
    got = np.array([oracle.round_half(x) for x in xs])
    want = xs.astype(np.float16).astype(np.float64)
    assert np.array_equal(got, want)


def test_half_network_matches_exact_network_on_binary16_values(oracle_lib):
    """With inputs, weights and every hidden activation exactly representable
    in binary16, the FP16 evaluation equals the exact one."""
    rng = np.random.default_rng(12)
    p = np.zeros(oracle.MLP_PARAMS)
    # integer inputs and hidden weights in {-1, 0, 1}: both hidden layers'
    # activations are integers below 2^11, exact in binary16
    p[0:224] = rng.integers(-1, 2, 224)
    p[224:1280] = rng.integers(-1, 2, 1056)
    p[1280:1313] = rng.normal(size=33)
    x = rng.integers(-2, 3, size=(300, 6)).astype(np.float64)
    assert np.array_equal(oracle.mlp_forward_half(p, x), oracle.mlp_forward(p, x))
    s1, s2, z = oracle.mlp_trace_half(p, x)
    assert np.all(s1 == np.round(s1)) and np.all(np.abs(s2) < 2048)
    assert np.allclose(1.0 / (1.0 + np.exp(-z)), oracle.mlp_forward(p, x), rtol=1e-15, atol=0)


def test_half_network_rounds_every_layer_input(oracle_lib):
    """A one-path network y = sigmoid(w3 relu(w2 relu(w1 x0))) : the FP16
    evaluation equals the exact network applied to x0 rounded to binary16, the
    first activation rounded to binary16 and the second activation rounded to
    binary16; the trace returns the two exact pre-activations."""
    p = np.zeros(oracle.MLP_PARAMS)
    w1, w2, w3 = 1.0 / 3.0, 0.7, 1.3
    p[0] = w1            # W1[0][0]
    p[224] = w2          # W2[0][0]
    p[1280] = w3         # W3[0]
    for x0 in (0.1, 1.2345, 3.14159, 7.3):
        x = np.zeros((1, 6))
        x[0, 0] = x0
        xh = float(np.float16(x0))
        h1 = float(np.float16(w1 * xh))
        h2 = float(np.float16(w2 * h1))
        want = 1.0 / (1.0 + np.exp(-(w3 * h2)))
        assert oracle.mlp_forward_half(p, x)[0] == pytest.approx(want, rel=1e-15)
        assert oracle.mlp_forward_half(p, x)[0] != oracle.mlp_forward(p, x)[0]
        # h2 rounding alone moves the output (the value without it differs)
        without_h2 = 1.0 / (1.0 + np.exp(-(w3 * (w2 * h1))))
        assert want != without_h2
        s1, s2, z = oracle.mlp_trace_half(p, x)
        assert s1[0, 0] == w1 * xh and s2[0, 0] == w2 * h1 and z[0] == w3 * h2
        # a negative pre-activation is clipped before rounding
        x[0, 0] = -x0
        assert oracle.mlp_forward_half(p, x)[0] == 0.5
