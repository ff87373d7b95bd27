"""Writes the stored oracle outputs under tests/golden/.  Calls only the oracle
and the seeded input generator; nothing here comes from the GPU library.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    oracle.build(force=False)
    g = synth.make_graph("T")
    pb = oracle.OracleProblem.from_synth(g)
    lin = pb.linearize(g.poses_init)
    P, st = pb.optimize(g.poses_init, 7)
    out = {
        "_about": "oracle on the tiny window (4 keyframes, 160x120, seed 0), 7 Gauss-Newton iterations",
        "poses_final": P.tolist(),
        "energy_f": st["energy_f"].tolist(),
        "energy_g": st["energy_g"].tolist(),
        "n_valid_g": st["n_valid_g"].tolist(),
        "n_valid_f": st["n_valid_f"].tolist(),
        "H0_diag": np.diag(lin["H"]).tolist(),
        "g0": lin["g"].tolist(),
    }
    with open(os.path.join(HERE, "oracle_tiny.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
