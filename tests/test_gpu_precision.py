"""GPU: the BF16x3 split-precision form of J^T W J (matrix-core products of
bf16 hi/lo splits accumulated in FP32; FP64 assembly, solve and update).

Bound: a product x_a x_b formed as hi_a hi_b + hi_a lo_b + lo_a hi_b drops
lo_a lo_b and inherits the two splitting errors, each at most 2^-16 of the
operand magnitude (bf16 keeps 8 significant bits, so |x - hi - lo| <=
2^-16 |x|), i.e. at most ~3 * 2^-16 = 4.6e-5 of |x_a x_b| per product.  Each
entry of H and g must therefore be within 5e-5 of the sum of magnitudes of
its contributions (plus the FP32 summation error), and the poses within
1e-4 rad / 1e-4 m of the FP64 oracle and of the plain FP32 GPU path."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import max_pose_diff

pytestmark = pytest.mark.gpu

SPLIT_BOUND = 5e-5


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


@pytest.mark.parametrize("name", ["T", "P"])
def test_bf16x3_normal_equations_within_split_bound(name):
    from paper_2108_00516_amd import _lib
    g = synth.make_graph(name)
    say(f"BF16x3 normal equations {name}")
    pg = gpu_graph(g, precision=_lib.PG_PREC_BF16X3)
    pb = oracle.OracleProblem.from_synth(g)
    dec = np.stack([pg.associate(i, j)[0] for (i, j) in pb.ordered_pairs()])
    lin = pb.linearize_given(g.poses_init, dec)
    H, gv, st = pg.linearize()
    dH = np.abs(H - lin["H"])
    fp32 = 1e-6 * np.abs(lin["H"]).max()
    assert np.all(dH <= SPLIT_BOUND * lin["H_abs"] + fp32), np.max(dH / (lin["H_abs"] + 1e-30))
    dg = np.abs(gv - lin["g"])
    assert np.all(dg <= SPLIT_BOUND * lin["g_abs"] + 1e-6 * lin["g_abs"].max())
    rel = np.linalg.norm(H - lin["H"]) / np.linalg.norm(lin["H"])
    say(f"  H rel Frobenius error {rel:.2e} (bound-limited)")
    assert st["n_valid_g"] == lin["n_valid_g"]
    assert st["energy_g"] == pytest.approx(lin["energy_g"], rel=1e-5)
    pg.close()


@pytest.mark.parametrize("name", ["P", "X"])
def test_bf16x3_poses(name):
    from paper_2108_00516_amd import _lib
    g = synth.make_graph(name)
    say(f"BF16x3 poses {name} ({g.n_frames} keyframes)")
    pb = gpu_graph(g, precision=_lib.PG_PREC_BF16X3)
    pb.optimize()
    pf = gpu_graph(g)
    pf.optimize()
    Po, _ = oracle.OracleProblem.from_synth(g).optimize(g.poses_init, 7)
    dr, dt = max_pose_diff(pb.poses, Po)
    dr2, dt2 = max_pose_diff(pb.poses, pf.poses)
    say(f"  vs oracle {dr:.2e} rad {dt:.2e} m; vs FP32 GPU {dr2:.2e} rad {dt2:.2e} m")
    assert dr <= 1e-4 and dt <= 1e-4
    assert dr2 <= 1e-4 and dt2 <= 1e-4
    pb.close()
    pf.close()
