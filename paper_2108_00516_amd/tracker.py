"""Causal object tracking with the keyframe memory pool (Sec. IV), built from
the library's GPU entry points: descriptor matching and RANSAC (Sec. IV-B),
keyframe selection (Sec. IV-C), the pose-graph optimisation (Sec. IV-D) and
the pool's augmentation (Sec. IV-E).  This module only sequences the calls
(argument marshalling and bookkeeping); every step runs in the library.

Per frame t with keypoints (pixel coordinates and descriptors), depth and
mask:
  1. the keypoints of frame t - 1 and t are matched and registered by RANSAC;
     the coarse pose is T~_t = T^-1 T_{t-1}, T the transform from frame t's
     camera to frame t - 1's;
  2. at most K keyframes are selected from the pool (the initial frame
     always) for T~_t;
  3. the graph of the selected keyframes and frame t is optimised: every pair
     of its nodes is matched and registered, each pair's RANSAC inliers become
     its feature matches (Eq. 2), the initial frame is held fixed;
  4. frame t's optimised pose is the output; the keyframes' corrected poses
     are written back to the pool (causal: earlier outputs are not revised);
  5. frame t joins the pool when its rotation is farther than 10 degrees from
     every keyframe's.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import frontend
from .posegraph import Camera, Config, PoseGraph


@dataclasses.dataclass
class Keyframe:
    index: int                 # frame index in the sequence
    depth: np.ndarray
    mask: np.ndarray
    uv: np.ndarray             # (n, 2) float32 keypoint pixel coordinates
    desc: np.ndarray           # (n, dim) float32 descriptors
    pose: np.ndarray           # (4, 4) current estimate (object -> camera)


class KeyframeTracker:
    def __init__(self, camera: Camera, K: int = 15, novel_deg: float = 10.0, config: Optional[Config] = None,
                 n_hyp: int = 256, delta: float = 0.005, alpha: float = float(np.deg2rad(45.0)),
                 ratio: float = 0.9, sample_fn=None):
        """sample_fn(frame_index, pair_index, n_matches, n_hyp) -> (n_hyp, 3)
        int32 match indices: the random draws of RANSAC (the caller's)."""
        self.camera = camera
        self.K = K
        self.novel_deg = novel_deg
        self.config = config or Config()
        self.n_hyp = n_hyp
        self.delta, self.alpha, self.ratio = delta, alpha, ratio
        self.sample_fn = sample_fn
        self.pool: List[Keyframe] = []
        self.prev: Optional[Keyframe] = None
        self.log: List[dict] = []

    def _graph(self, frames, poses, n_nodes):
        cfg = dataclasses.replace(self.config, max_frames=max(n_nodes, 2))
        pg = PoseGraph(self.camera, cfg)
        for k, (f, T) in enumerate(zip(frames, poses)):
            pg.add_frame(f.depth, f.mask, T, fixed=(k == 0 and f.index == 0))
        return pg

    def _match_pairs(self, frames, pairs):
        import torch
        sets = [np.ascontiguousarray(f.desc, np.float32) for f in frames]
        off = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int32)
        desc = torch.from_numpy(np.concatenate(sets, axis=0)).cuda()
        m, _, _ = frontend.match_descriptors(desc, off, pairs, self.ratio, with_distances=False)
        m = m.cpu().numpy()
        out, o = [], 0
        for a, b in pairs:
            mm = m[o:o + len(sets[a])]
            o += len(sets[a])
            src = np.flatnonzero(mm >= 0)
            out.append((frames[a].uv[src], frames[b].uv[mm[src]]))
        return out

    def _samples(self, t, q, n):
        return self.sample_fn(t, q, n, self.n_hyp)

    def step(self, t: int, depth, mask, uv, desc, init_pose=None) -> np.ndarray:
        """Track frame t; returns its pose (object -> camera).  The first
        frame needs init_pose (the reference, held fixed from then on)."""
        cur = Keyframe(t, depth, mask, np.asarray(uv, np.float32), np.asarray(desc, np.float32), np.eye(4))
        if not self.pool:
            # the initial frame: the reference pose, the first keyframe
            if init_pose is None:
                raise ValueError("the first frame needs its pose")
            cur.index = 0
            cur.pose = np.asarray(init_pose, np.float64)
            self.pool.append(cur)
            self.prev = cur
            self.log.append(dict(t=t, selected=[], novel=True, coarse=cur.pose))
            return cur.pose
        # 1. coarse pose from RANSAC against the previous frame
        prev = self.prev
        (ui, uj), = self._match_pairs([prev, cur], [(0, 1)])
        pg = self._graph([prev, cur], [prev.pose, prev.pose], 2)
        reg = pg.ransac([(0, 1)], [ui], [uj], self._samples(t, 0, len(ui)).reshape(1, -1, 3), self.delta,
                        self.alpha)
        pg.close()
        coarse = np.linalg.inv(reg["T"][0]) @ prev.pose if reg["best"][0] >= 0 else prev.pose
        # 2. keyframes for the coarse pose
        sel, _, _ = frontend.select_keyframes(np.stack([k.pose for k in self.pool]), coarse, self.K,
                                              self.novel_deg)
        nodes = [self.pool[s] for s in sel] + [cur]
        # 3. the window graph: every pair matched, registered, inliers installed
        pairs = [(i, j) for i in range(len(nodes)) for j in range(i + 1, len(nodes))]
        mt = self._match_pairs(nodes, pairs)
        poses = [n.pose for n in nodes[:-1]] + [coarse]
        pg = self._graph(nodes, poses, len(nodes))
        samples = np.stack([self._samples(t, 1 + q, len(a)) for q, (a, _) in enumerate(mt)])
        pg.ransac(pairs, [a for a, _ in mt], [b for _, b in mt], samples, self.delta, self.alpha, install=True)
        st = pg.optimize(check=False)
        P = pg.poses if st["status"] == 0 else np.stack(poses)
        pg.close()
        # 4. output and write-back
        for s, T in zip(sel, P[:-1]):
            if self.pool[s].index != 0:
                self.pool[s].pose = T
        cur.pose = P[-1]
        # 5. the pool grows with novel views
        _, novel, _ = frontend.select_keyframes(np.stack([k.pose for k in self.pool]), cur.pose, 1,
                                                self.novel_deg)
        if novel:
            self.pool.append(cur)
        self.prev = cur
        self.log.append(dict(t=t, selected=[self.pool[s].index for s in sel], novel=novel, coarse=coarse,
                             status=st["status"]))
        return cur.pose
