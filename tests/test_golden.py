"""Stored values: the paper's constants (cited) and a regression record of the
oracle on the tiny window (written by tests/golden/make_golden.py)."""
import json
import os

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_method_constants_follow_the_paper():
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    p = oracle.Params()
    assert p.lambda_f == c["lambda_1"]["value"] and p.lambda_g == c["lambda_2"]["value"]
    # Huber thresholds read as the paper's inlier distance scale
    assert p.huber_f == c["ransac_inlier_distance_m"]["value"] == p.huber_g


def test_oracle_regression_tiny(oracle_lib):
    ref = json.load(open(os.path.join(GOLDEN, "oracle_tiny.json")))
    g = synth.make_graph("T")
    pb = oracle.OracleProblem.from_synth(g)
    P, st = pb.optimize(g.poses_init, 7)
    assert np.allclose(P, np.array(ref["poses_final"]), rtol=0, atol=1e-12)
    assert np.allclose(st["energy_g"], ref["energy_g"], rtol=1e-12)
    assert list(st["n_valid_g"]) == ref["n_valid_g"]
