"""Oracle pins on the assembled normal equations and the whole Gauss-Newton
iteration: symmetry/PSD, the gauge null space of the dense term, the feature
gradient against finite differences of the energy, recovery of known poses,
the Arun/Umeyama closed form, a brute-force local-minimum check, failure codes
and thread-count independence."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth


def adjoint(T):
    R, t = T[:3, :3], T[:3, 3]
    tx = np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])
    A = np.zeros((6, 6))
    A[:3, :3] = R
    A[:3, 3:] = tx @ R
    A[3:, 3:] = R
    return A


@pytest.fixture(scope="module")
def graph_t():
    return synth.make_graph("T")


def test_H_symmetric_psd(oracle_lib, graph_t):
    lin = oracle.OracleProblem.from_synth(graph_t).linearize(graph_t.poses_init)
    H = lin["H"]
    assert np.array_equal(H, H.T)
    ev = np.linalg.eigvalsh(H)
    assert ev.min() >= -1e-12 * np.abs(H).max()


def test_dense_term_gauge_null_space(oracle_lib, graph_t):
    # E_g depends on T_i T_j^-1 only: moving every pose by the same object-frame
    # twist z (T_i -> T_i Exp(z) = Exp(Ad_{T_i} z) T_i) leaves it unchanged
    pb = oracle.OracleProblem.from_synth(graph_t, oracle.Params(lambda_f=0.0))
    P = graph_t.poses_init
    lin = pb.linearize(P)
    H, g = lin["H"], lin["g"]
    for k in range(6):
        z = np.zeros(6)
        z[k] = 1.0
        v = np.concatenate([adjoint(P[i]) @ z for i in range(graph_t.n_frames)])
        assert np.linalg.norm(H @ v) <= 1e-10 * np.linalg.norm(H) * np.linalg.norm(v)
        assert abs(g @ v) <= 1e-10 * np.abs(lin["g_abs"]).sum() * np.linalg.norm(v)


def test_feature_gradient_finite_difference(oracle_lib, graph_t):
    pb = oracle.OracleProblem.from_synth(graph_t, oracle.Params(lambda_g=0.0))
    P = graph_t.poses_init
    lin = pb.linearize(P)
    h = 1e-6
    for node in range(graph_t.n_frames):
        for k in range(6):
            xi = np.zeros(6)
            xi[k] = h
            Pp, Pm = P.copy(), P.copy()
            Pp[node] = oracle.se3_exp(xi) @ P[node]
            Pm[node] = oracle.se3_exp(-xi) @ P[node]
            fd = (pb.linearize(Pp)["energy_f"] - pb.linearize(Pm)["energy_f"]) / (2 * h)
            assert abs(fd - lin["g"][6 * node + k]) < 1e-6 * lin["g_abs"].max()


def _identical_window(n=4, clean=True):
    """n copies of one rendered frame at one pose: exact correspondences."""
    g = synth.make_graph("T", noise_sigma=0.0)
    depth = np.repeat(g.depth[1][None], n, 0)
    mask = np.repeat(g.mask[1][None], n, 0)
    gt = np.repeat(g.poses_gt[1][None], n, 0)
    rng = np.random.default_rng(5)
    vv, uu = np.nonzero(g.mask[1])
    matches = []
    for i in range(n):
        for j in range(i + 1, n):
            sel = rng.choice(len(uu), 40, replace=False)
            uv = np.stack([uu[sel], vv[sel]], 1).astype(np.float32)
            matches.append(synth.MatchSet(i, j, uv, uv.copy(), np.ones(40, bool)))
    init = gt.copy()
    for k in range(1, n):
        init[k] = synth.perturb_pose(rng, gt[k], np.deg2rad(1.0), 0.005)
    return g, depth, mask, gt, init, matches


@pytest.mark.parametrize("terms", ["f", "g", "fg"])
def test_exact_recovery_identical_frames(oracle_lib, terms):
    g, depth, mask, gt, init, matches = _identical_window()
    prm = oracle.Params(lambda_f=1.0 if "f" in terms else 0.0, lambda_g=1.0 if "g" in terms else 0.0)
    fixed = np.array([1, 0, 0, 0], np.int32)
    pb = oracle.OracleProblem(depth, mask, g.fx, g.fy, g.cx, g.cy, fixed, matches, prm)
    P, st = pb.optimize(init, 12)
    assert st["status"] == oracle.OK
    for k in range(4):
        ra, ta = oracle.pose_error(P[k], gt[k])
        assert ra < 1e-9 and ta < 1e-9, (terms, k, ra, ta)
    E = st["energy_f"] + st["energy_g"]
    assert E[-1] < 1e-18


def test_arun_umeyama_two_nodes(oracle_lib):
    # 2 nodes, feature term only, no robust cut-off: the minimiser over T_1 of
    # sum |T_0^-1 p_m - T_1^-1 p_n|^2 is the least-squares rigid alignment of
    # the points p_n onto a_m = T_0^-1 p_m (Arun et al.; SVD).
    g = synth.make_graph("T", outlier_frac=0.0, n_frames=2)
    prm = oracle.Params(lambda_g=0.0, huber_f=1e6)
    pb = oracle.OracleProblem.from_synth(g, prm)
    P, st = pb.optimize(g.poses_init, 25)
    assert st["status"] == oracle.OK
    m = g.matches[0]
    V0, _, _ = pb.preprocess(0)
    V1, _, _ = pb.preprocess(1)
    r = lambda uv: np.floor(uv.astype(np.float64) + 0.5).astype(int)
    ui, uj = r(m.uv_i), r(m.uv_j)
    pm = V0[ui[:, 1], ui[:, 0]]
    pn = V1[uj[:, 1], uj[:, 0]]
    T0inv = np.linalg.inv(g.poses_init[0])
    a = pm @ T0inv[:3, :3].T + T0inv[:3, 3]
    b = pn
    ca, cb = a.mean(0), b.mean(0)
    U, S, Vt = np.linalg.svd((b - cb).T @ (a - ca))
    D = np.diag([1, 1, np.sign(np.linalg.det(Vt.T @ U.T))])
    R = Vt.T @ D @ U.T               # maps b onto a
    t = ca - R @ cb
    Sinv = np.eye(4)
    Sinv[:3, :3], Sinv[:3, 3] = R, t  # = T_1^-1
    T1 = np.linalg.inv(Sinv)
    ra, ta = oracle.pose_error(P[1], T1)
    assert ra < 1e-9 and ta < 1e-9, (ra, ta)


def test_recovers_ground_truth_clean(oracle_lib):
    g = synth.make_graph("T", noise_sigma=0.0, outlier_frac=0.0)
    pb = oracle.OracleProblem.from_synth(g)
    P, st = pb.optimize(g.poses_init, 10)
    assert st["status"] == oracle.OK
    e0 = max(oracle.pose_error(g.poses_init[k], g.poses_gt[k])[0] for k in range(4))
    errs = [oracle.pose_error(P[k], g.poses_gt[k]) for k in range(4)]
    # discretisation floor of nearest-pixel association and sub-pixel matches at 160x120
    assert max(e[0] for e in errs) < 5e-3 < e0 * 2
    assert max(e[1] for e in errs) < 1e-3
    E = st["energy_f"] + st["energy_g"]
    assert E[-1] < E[0]


def test_converged_point_is_a_local_minimum(oracle_lib):
    # at convergence, no +-1e-6 step of a free coordinate lowers the energy
    # (association re-decided at each probe, as the method does)
    g = synth.make_graph("T", width=80, height=60, n_frames=3)
    pb = oracle.OracleProblem.from_synth(g)
    P, st = pb.optimize(g.poses_init, 20)
    lin = pb.linearize(P)
    E0 = lin["energy_f"] + lin["energy_g"]
    for node in (1, 2):
        for k in range(6):
            for s in (1e-6, -1e-6):
                xi = np.zeros(6)
                xi[k] = s
                Q = P.copy()
                Q[node] = oracle.se3_exp(xi) @ P[node]
                l2 = pb.linearize(Q)
                assert l2["energy_f"] + l2["energy_g"] >= E0 - 1e-12 * E0


def test_singular_node_reports_error_and_keeps_poses(oracle_lib):
    g = synth.make_graph("T")
    mask = g.mask.copy()
    mask[2] = 0                       # node 2 sees nothing
    matches = [m for m in g.matches if 2 not in (m.i, m.j)]
    pb = oracle.OracleProblem(g.depth, mask, g.fx, g.fy, g.cx, g.cy, g.fixed, matches)
    P, st = pb.optimize(g.poses_init, 7)
    assert st["status"] == oracle.ERR_SINGULAR
    assert st["iters_done"] == 0
    assert np.array_equal(P, g.poses_init)


def test_all_fixed_is_a_no_op(oracle_lib, graph_t):
    pb = oracle.OracleProblem(graph_t.depth, graph_t.mask, graph_t.fx, graph_t.fy, graph_t.cx, graph_t.cy,
                              np.ones(4, np.int32), graph_t.matches)
    P, st = pb.optimize(graph_t.poses_init, 3)
    assert st["status"] == oracle.OK and st["iters_done"] == 3
    assert np.array_equal(P, graph_t.poses_init)


def test_threads_do_not_change_results(oracle_lib, graph_t):
    pb = oracle.OracleProblem.from_synth(graph_t)
    oracle.set_threads(1)
    P1, s1 = pb.optimize(graph_t.poses_init, 4)
    oracle.set_threads(4)
    P4, s4 = pb.optimize(graph_t.poses_init, 4)
    oracle.set_threads(1)
    assert np.array_equal(P1, P4)
    assert np.array_equal(s1["energy_g"], s4["energy_g"])


def test_linearize_given_own_decisions_is_identical(oracle_lib, graph_t):
    # fed the oracle's own association decisions, the given-decision entry
    # reproduces orc_linearize bit for bit
    pb = oracle.OracleProblem.from_synth(graph_t)
    P = graph_t.poses_init
    tg = np.stack([pb.associate(P, i, j)[0] for (i, j) in pb.ordered_pairs()])
    a = pb.linearize(P)
    b = pb.linearize_given(P, tg)
    for k in ("H", "g", "H_abs", "g_abs"):
        assert np.array_equal(a[k], b[k]), k
    assert a["energy_g"] == b["energy_g"] and a["n_valid_g"] == b["n_valid_g"]
    # dropping one decision removes exactly that residual's contribution
    i, j = pb.ordered_pairs()[0]
    x = np.flatnonzero(tg[0] >= 0)[0]
    tg2 = tg.copy()
    tg2[0, x] = -1
    c = pb.linearize_given(P, tg2)
    assert c["n_valid_g"] == a["n_valid_g"] - 1
    r, J = pb.dense_frozen(P, i, j, [x], [tg[0, x]])
    w = oracle.huber_weight(abs(r[0]), pb.params.huber_g)
    idx = np.r_[6 * i:6 * i + 6, 6 * j:6 * j + 6]
    dH = np.zeros_like(a["H"])
    dH[np.ix_(idx, idx)] = w * np.outer(J[0], J[0])
    assert np.allclose(a["H"] - c["H"], dH, atol=1e-9 * np.abs(a["H"]).max())
