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
            config: Optional[Config] = None):
    """Samples of (features (n, 6), labels (n,)) as float32 device tensors.

    windows: (SynthGraph with leaky masks, reference poses (N, 4, 4)).
    Features are taken at the first `iters` iterates of the plain optimiser."""
    import torch
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
        # reference association per ordered pair
        fg.set_poses(ref)
        good = {}
        for (i, j) in _pairs(g.n_frames):
            fg.pair_features(i, j, 0, out=(f, None, t))
            good[(i, j)] = (t >= 0) & (f[:, 0].abs() * cfg.huber_g_m < inlier_m)
        P = np.array(g.poses_init)
        for k in range(iters):
            fg.set_poses(P)
            for (i, j) in _pairs(g.n_frames):
                fg.pair_features(i, j, k, out=(f, None, t))
                sel = t >= 0
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
