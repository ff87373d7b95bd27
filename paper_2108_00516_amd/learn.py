"""Training data and training of the learned correspondence weighting.

Labels come from the plain (Huber-weighted) optimiser: for a window whose
masks leak onto the background, the reference poses are those the plain
optimiser reaches on the same frames with their true masks.  A dense
pixel-pair of the leaky window, taken at any iterate of the plain optimiser on
it, is labelled 1 when its source pixel, at the reference poses, is gated in
to the same target frame with a point-to-plane residual under `inlier_m`, and
0 otherwise.  Features are the library's own (pose_graph_pair_features), so
the network is trained on exactly what the association kernels feed it.

Every step runs through the library: feature extraction and the optimiser
iterations in the association kernels, the loss, gradient and Adam update in
the trainer kernels.  torch only holds the device buffers and shuffles sample
indices.
"""
from __future__ import annotations

from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib as L
from .posegraph import Config, MlpTrainer, from_synth

N_PARAMS = 1313


def init_params(seed: int = 0) -> np.ndarray:
    """He-initialised parameters (zero biases, output bias 1: weights start
    near sigmoid(1) = 0.73 everywhere), float32."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS, np.float32)
    p[0:192] = rng.normal(0.0, np.sqrt(2.0 / 6.0), 192)
    p[224:1248] = rng.normal(0.0, np.sqrt(2.0 / 32.0), 1024)
    p[1280:1312] = rng.normal(0.0, np.sqrt(1.0 / 32.0), 32)
    p[1312] = 1.0
    return p


def _pairs(n: int) -> List[Tuple[int, int]]:
    return [(i, j) for i in range(n) for j in range(n) if i != j]


def collect(windows: Iterable[Tuple[object, np.ndarray]], iters: int = 7, inlier_m: float = 0.003,
            config: Optional[Config] = None, sample_frac: float = 1.0, seed: int = 0, max_pairs: int = 0):
    """Samples of (features (n, 6), labels (n,)) as float32 device tensors.

    windows: (SynthGraph with leaky masks, reference poses (N, 4, 4)).
    Features are taken at the first `iters` iterates of the plain optimiser;
    sample_frac < 1 keeps a seeded random subset of each pair's samples;
    max_pairs > 0 takes a seeded subset of that many ordered pairs of a larger
    window (the same pairs at every iterate)."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    feats, labels = [], []
    base = config or Config()
    for g, ref in windows:
        cfg = Config(**{**base.__dict__, "max_frames": max(g.n_frames, 2), "gn_iters": iters,
                        "weighting": L.PG_WEIGHT_HUBER})
        step_cfg = Config(**{**cfg.__dict__, "gn_iters": 1})
        fg = from_synth(g, cfg, device_inputs=True)       # feature extraction (iteration normaliser)
        sg = from_synth(g, step_cfg, device_inputs=True)  # one plain iteration per call
        hw = g.width * g.height
        f = torch.empty((hw, 6), dtype=torch.float32, device="cuda")
        t = torch.empty(hw, dtype=torch.int32, device="cuda")
        pairs = _pairs(g.n_frames)
        if 0 < max_pairs < len(pairs):
            pick = np.random.default_rng([seed, g.n_frames, 17]).choice(len(pairs), max_pairs, replace=False)
            pairs = [pairs[q] for q in sorted(pick)]
        # reference association per ordered pair
        fg.set_poses(ref)
        good = {}
        for (i, j) in pairs:
            fg.pair_features(i, j, 0, out=(f, None, t))
            good[(i, j)] = (t >= 0) & (f[:, 0].abs() * cfg.huber_g_m < inlier_m)
        P = np.array(g.poses_init)
        for k in range(iters):
            fg.set_poses(P)
            for (i, j) in pairs:
                fg.pair_features(i, j, k, out=(f, None, t))
                sel = t >= 0
                if sample_frac < 1.0:
                    sel &= torch.rand(hw, device="cuda", generator=gen) < sample_frac
                feats.append(f[sel].clone())
                labels.append(good[(i, j)][sel].float())
            sg.set_poses(P)
            sg.optimize(check=False)
            P = sg.poses
        fg.close()
        sg.close()
    return torch.cat(feats), torch.cat(labels)


def train(x, y, steps: int = 400, lr: float = 3e-3, batch: int = 65536, seed: int = 0,
          params: Optional[np.ndarray] = None, log=None) -> Tuple[np.ndarray, MlpTrainer]:
    """Adam on the mean binary cross-entropy over shuffled minibatches.
    Returns (fp16 parameters, trainer)."""
    import torch
    n = x.shape[0]
    batch = min(batch, n)
    tr = MlpTrainer(batch)
    tr.set_params(init_params(seed) if params is None else params)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    perm = torch.randperm(n, device="cuda", generator=gen)
    pos = 0
    for s in range(steps):
        if pos + batch > n:
            perm = torch.randperm(n, device="cuda", generator=gen)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        xb = x[idx].contiguous()
        yb = y[idx].contiguous()
        want = log is not None and (s % 50 == 0 or s == steps - 1)
        loss = tr.adam_step(xb, yb, lr, want_loss=want)
        if want:
            log(f"step {s}: batch loss {loss:.4f}")
    return tr.params_fp16(), tr


def reference_poses(g_clean, config: Optional[Config] = None) -> np.ndarray:
    """Poses of the plain optimiser on a window with its true masks."""
    cfg = config or Config(max_frames=max(g_clean.n_frames, 2))
    pg = from_synth(g_clean, cfg, device_inputs=True)
    pg.optimize(check=False)
    P = pg.poses
    pg.close()
    return P


def _training_window(k: int, large_every: int = 0):
    """k-th training window (seed 10000 + k) with its true masks and with
    masks grown by k mod 6 pixels: the 20-keyframe 640x480 shape ('L') for
    every large_every-th k (none for 0), else a 4-keyframe 160x120 scene."""
    import synth
    seed = 10_000 + k
    preset = "L" if large_every > 0 and k % large_every == 0 else "T"
    return synth.make_graph(preset, seed=seed), synth.make_graph(preset, seed=seed, mask_dilate=k % 6)


def _evaluation_window(k: int):
    """k-th evaluation window (seed 20000 + k, held out from training), masks
    grown by 4 pixels: the 10-keyframe 640x480 shape for every 5th k, else a
    4-keyframe 160x120 scene."""
    import synth
    return synth.make_graph("P" if k % 5 == 0 else "T", seed=20_000 + k, mask_dilate=4)


def pose_error_rad(Ta: np.ndarray, Tb: np.ndarray) -> float:
    """Rotation angle between two poses' rotations (radians)."""
    c = (np.trace(Ta[:3, :3] @ Tb[:3, :3].T) - 1.0) / 2.0
    return float(np.arccos(np.clip(c, -1.0, 1.0)))


def evaluate(p16: np.ndarray, n: int = 100, workers: int = 16, prune_frac: float = 0.25, log=print) -> dict:
    """Plain and learned optimisation of the held-out windows of seeds 20000 ..
    20000 + n - 1: per window shape, the mean and median over the windows of
    each form's largest rotation error against the ground truth, of the
    learned form's largest pose difference to the plain one, and the count of
    windows where the learned form is closer to the ground truth."""
    import multiprocessing as mp
    import os

    import torch

    from . import _lib as L2
    res = {}
    with mp.get_context("fork").Pool(max(1, min(workers, os.cpu_count() or 1))) as pool:
        torch.cuda.set_device(0)
        for g in pool.imap(_evaluation_window, range(n), chunksize=2):
            out = {}
            for kind in ("plain", "learned"):
                cfg = Config(max_frames=g.n_frames)
                if kind == "learned":
                    cfg = Config(max_frames=g.n_frames, weighting=L2.PG_WEIGHT_LEARNED, prune_frac=prune_frac)
                pg = from_synth(g, cfg, device_inputs=True)
                if kind == "learned":
                    pg.set_mlp(p16)
                pg.optimize(check=False)
                out[kind] = pg.poses
                pg.close()
            e = {k: max(pose_error_rad(out[k][f], g.poses_gt[f]) for f in range(g.n_frames)) for k in out}
            d = max(pose_error_rad(out["learned"][f], out["plain"][f]) for f in range(g.n_frames))
            r = res.setdefault(f"{g.n_frames} keyframes {g.width}x{g.height}", {"plain": [], "learned": [], "diff": []})
            r["plain"].append(e["plain"])
            r["learned"].append(e["learned"])
            r["diff"].append(d)
            if log and sum(len(v["plain"]) for v in res.values()) % 20 == 0:
                log(f"evaluated {sum(len(v['plain']) for v in res.values())} windows")
    summary = {}
    for shape, r in res.items():
        pl, le, di = (np.array(r[k]) for k in ("plain", "learned", "diff"))
        summary[shape] = {"windows": int(len(pl)),
                          "plain_rot_err_rad": {"mean": float(pl.mean()), "median": float(np.median(pl))},
                          "learned_rot_err_rad": {"mean": float(le.mean()), "median": float(np.median(le))},
                          "learned_vs_plain_rad": {"mean": float(di.mean()), "max": float(di.max())},
                          "learned_closer": int((le < pl).sum())}
        if log:
            log(f"{shape}: {summary[shape]}")
    return summary


def main(argv=None):
    """Train the weighting network on seeded synthetic windows and write its
    fp16 parameters (.npy) and a record of the run (.json)."""
    import argparse
    import json
    import multiprocessing as mp
    import os
    import time

    import torch
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--graphs", type=int, default=10_000)
    ap.add_argument("--sample-frac", type=float, default=0.02)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", required=True, help="output .npy (fp16 parameters)")
    ap.add_argument("--evaluate", type=int, default=100, help="held-out evaluation windows (0: none)")
    ap.add_argument("--large-every", type=int, default=0,
                    help="every n-th training window has the 20-keyframe 640x480 shape (0: none)")
    ap.add_argument("--log-every", type=int, default=100)
    a = ap.parse_args(argv)
    t0 = time.time()
    xs, ys = [], []
    # the workers only build scenes on the CPU; they are forked before this
    # process touches the GPU
    with mp.get_context("fork").Pool(max(1, min(a.workers, os.cpu_count() or 1))) as pool:
        torch.cuda.set_device(0)
        done = 0
        import functools
        window = functools.partial(_training_window, large_every=a.large_every)
        for clean, leaky in pool.imap(window, range(a.graphs), chunksize=8):
            ref = reference_poses(clean)
            x, y = collect([(leaky, ref)], sample_frac=a.sample_frac, seed=a.seed + done, max_pairs=40)
            xs.append(x)
            ys.append(y)
            done += 1
            if done % a.log_every == 0 or clean.n_frames > 4:
                print(f"{done} windows ({clean.n_frames} keyframes last), {sum(len(v) for v in ys)} samples, "
                      f"{time.time() - t0:.0f} s", flush=True)
    x, y = torch.cat(xs), torch.cat(ys)
    t1 = time.time()
    p16, tr = train(x, y, steps=a.steps, lr=a.lr, batch=a.batch, seed=a.seed,
                    log=lambda m: print(m, flush=True))
    m = min(len(y), a.batch)
    loss, _ = tr.loss_grad(x[:m].contiguous(), y[:m].contiguous())
    tr.close()
    np.save(a.out, p16, allow_pickle=False)
    rec = dict(graphs=a.graphs, samples=int(len(y)), inlier_fraction=float(y.mean()), steps=a.steps, lr=a.lr,
               batch=a.batch, seed=a.seed, sample_frac=a.sample_frac, final_loss_first_batch=loss,
               collect_s=round(t1 - t0, 1), train_s=round(time.time() - t1, 1),
               windows="4 keyframes 160x120 (seeds 10000..), masks grown by k mod 6 px; labels: gated in "
                       "with |r| < 3 mm at the plain optimiser's poses on the true masks")
    large = len(range(0, a.graphs, a.large_every)) if a.large_every > 0 else 0
    shapes = (f"{large} of 20 keyframes 640x480 (every {a.large_every}th, 40 seeded ordered pairs each), the rest "
              "4 keyframes 160x120" if large else "4 keyframes 160x120")
    rec["windows"] = (f"seeds 10000..{10_000 + a.graphs - 1}: {shapes}; masks grown by k mod 6 px; labels: gated "
                      "in with |r| < 3 mm at the plain optimiser's poses on the true masks")
    rec["large_windows"] = large
    if a.evaluate > 0:
        rec["evaluation"] = {"seeds": f"20000..{20_000 + a.evaluate - 1} (every 5th 10 keyframes 640x480, the rest "
                                      "4 keyframes 160x120; masks grown by 4 px), prune 25 %",
                             "results": evaluate(p16, a.evaluate, a.workers)}
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
