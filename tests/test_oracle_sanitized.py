"""The CPU checker under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle.c is built with -fsanitize=address,undefined (every finding fatal) and
every entry point is exercised on small seeded inputs in a child process that
preloads the ASan runtime: plain and learned optimisation (with pruning),
linearisation (own and given decisions), association, frozen dense terms,
feature terms, the network (FP64, binary16, traces, loss and gradient),
pruning scores and selection, RANSAC registration and descriptor matching.
A finding aborts the child with the sanitizer's report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
import oracle, synth
oracle.set_threads(2)
g = synth.make_graph("T", n_frames=3, width=48, height=36, n_matches=20)
pb = oracle.OracleProblem.from_synth(g)
P, st = pb.optimize(g.poses_init, 2)
assert st["iters_done"] == 2
pb.linearize(g.poses_init)
for f in range(g.n_frames):
    pb.preprocess(f)
for (i, j) in pb.ordered_pairs()[:3]:
    a = pb.associate(g.poses_init, i, j)
rng = np.random.default_rng(0)
params = rng.standard_normal(1313) * 0.1
x = rng.standard_normal((17, 6))
oracle.mlp_forward(params, x)
oracle.mlp_forward_half(params, x)
oracle.mlp_trace_half(params, x)
oracle.mlp_bce(params, x, (rng.random(17) > 0.5).astype(np.float64))
pl = oracle.OracleProblem.from_synth(g, oracle.Params(mlp=params, prune_frac=0.25))
sc = pl.prune_scores(g.poses_init)
keep = pl.prune_select(sc, 0.25)
pl.pair_features(g.poses_init, 0, 1)
pl.optimize(g.poses_init, 2)
oracle.se3_exp(rng.standard_normal(6) * 0.1)
A = rng.standard_normal((6, 8)); oracle.cholesky_solve(A @ A.T, rng.standard_normal(6))
pts = rng.standard_normal((10, 3)); oracle.arun(pts, pts + 0.01)
m = g.matches[0]
samples = synth.ransac_samples(0, len(m.uv_i), 8)
pb.ransac([(m.i, m.j)], [m.uv_i], [m.uv_j], samples.reshape(1, -1, 3), scores=True)
D = rng.standard_normal((12, 16)).astype(np.float32)
oracle.match_descriptors(D, D[::-1].copy(), ratio=0.8)
print("SANITIZED_OK", flush=True)
"""


def test_oracle_under_asan_and_ubsan(tmp_path):
    import oracle
    lib = oracle.build(force=True, sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no ASan runtime for gcc")
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, cwd=str(tmp_path), capture_output=True,
                       text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "SANITIZED_OK" in r.stdout, tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
