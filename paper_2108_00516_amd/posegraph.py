"""Python binding of the pose-graph library: argument marshalling only.

Every step of the optimisation runs in the HIP kernels behind the C ABI.
Frames may be given as NumPy arrays (host memory) or torch tensors (host or
device); torch supplies device memory and the stream, nothing else.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

from . import _lib as L


class PoseGraphError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {message}")


@dataclasses.dataclass
class Config:
    """Mirror of pg_config (defaults as pg_config_default)."""
    max_frames: int = 16
    gn_iters: int = 7
    lambda_f: float = 1.0
    lambda_g: float = 1.0
    huber_f_m: float = 0.005
    huber_g_m: float = 0.005
    gate_dist_m: float = 0.01
    gate_normal_rad: float = math.radians(30.0)
    solver: int = L.PG_SOLVER_AUTO
    pcg_max_iters: int = 500
    pcg_rel_tol: float = 1e-12
    weighting: int = L.PG_WEIGHT_HUBER
    precision: int = L.PG_PREC_FP32
    use_graph: int = 0
    timing: int = 0
    tile_pixels: int = 0
    prune_frac: float = 0.25
    persistent: int = 0

    def to_c(self) -> L.pg_config:
        c = L.pg_config()
        for f in dataclasses.fields(self):
            setattr(c, f.name, getattr(self, f.name))
        return c


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def to_c(self) -> L.pg_camera:
        return L.pg_camera(self.width, self.height, self.fx, self.fy, self.cx, self.cy)


def stats_to_dict(s: L.pg_stats, iters: int) -> dict:
    k = max(0, min(iters, L.PG_MAX_ITERS))
    return dict(iters_done=s.iters_done, energy_f=np.array(s.energy_f[:k]), energy_g=np.array(s.energy_g[:k]),
                n_valid_g=np.array(s.n_valid_g[:k]), n_valid_f=np.array(s.n_valid_f[:k]),
                n_target_reads=np.array(s.n_target_reads[:k]), pcg_iters=np.array(s.pcg_iters[:k]),
                status_bits=s.status_bits, src_pixels=s.src_pixels, n_assoc_launches=s.n_assoc_launches,
                ms_assoc=s.ms_assoc, ms_feature=s.ms_feature, ms_reduce=s.ms_reduce, ms_solve=s.ms_solve,
                ms_total=s.ms_total)


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return C.c_void_p(None)


def _pointer(a, dtype, shape):
    """(pointer, keep-alive) of an array-like with the given dtype and shape:
    torch tensors (host or device) are passed by their data pointer, anything
    else through a contiguous NumPy copy in host memory."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            tdt = {np.float32: torch.float32, np.uint8: torch.uint8}[dtype]
            t = a.detach().to(tdt).contiguous()
            if tuple(t.shape) != tuple(shape):
                raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
            return C.c_void_p(t.data_ptr()), t
    except ImportError:
        pass
    arr = np.ascontiguousarray(a, dtype=dtype)
    if arr.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {arr.shape}")
    return C.c_void_p(arr.ctypes.data), arr


class PoseGraph:
    """One keyframe window on the GPU (pose_graph_* handle)."""

    def __init__(self, camera: Camera, config: Optional[Config] = None, stream=None):
        self.lib = L.load()
        self.camera = camera
        self.config = config or Config()
        self._cfg = self.config.to_c()
        self._cam = camera.to_c()
        if stream is None:
            st = _current_stream()
        elif isinstance(stream, int):
            st = C.c_void_p(stream)
        else:
            st = C.c_void_p(stream.cuda_stream)
        self._stream = st
        h = C.c_void_p()
        rc = self.lib.pose_graph_create(C.byref(self._cfg), C.byref(self._cam), st, C.byref(h))
        if rc != L.PG_OK:
            raise PoseGraphError(rc, self.lib.pose_graph_last_error(None).decode())
        self.h = h

    # ------------------------------------------------------------ helpers
    def _check(self, rc):
        if rc != L.PG_OK:
            raise PoseGraphError(rc, self.lib.pose_graph_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.pose_graph_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def n_frames(self) -> int:
        return self.lib.pose_graph_num_frames(self.h)

    # -------------------------------------------------------- entry points
    def add_frame(self, depth, mask, T, fixed: bool = False) -> int:
        H, W = self.camera.height, self.camera.width
        dp, keep_d = _pointer(depth, np.float32, (H, W))
        mp, keep_m = _pointer(mask, np.uint8, (H, W))
        Tm = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        out = C.c_int()
        self._check(self.lib.pose_graph_add_frame(self.h, dp, mp, Tm.ctypes.data_as(C.POINTER(C.c_double)),
                                                  int(bool(fixed)), C.byref(out)))
        return out.value

    def add_matches(self, i: int, j: int, uv_i, uv_j):
        n = int(np.asarray(uv_i.shape[0] if hasattr(uv_i, "shape") else len(uv_i)))
        if n == 0:
            self._check(self.lib.pose_graph_add_matches(self.h, i, j, None, None, 0))
            return
        a, ka = _pointer(uv_i, np.float32, (n, 2))
        b, kb = _pointer(uv_j, np.float32, (n, 2))
        self._check(self.lib.pose_graph_add_matches(self.h, i, j, a, b, n))

    def set_pose(self, i: int, T):
        Tm = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        self._check(self.lib.pose_graph_set_pose(self.h, i, Tm.ctypes.data_as(C.POINTER(C.c_double))))

    def get_pose(self, i: int) -> np.ndarray:
        T = np.zeros(16)
        self._check(self.lib.pose_graph_get_pose(self.h, i, T.ctypes.data_as(C.POINTER(C.c_double))))
        return T.reshape(4, 4)

    @property
    def poses(self) -> np.ndarray:
        return np.stack([self.get_pose(i) for i in range(self.n_frames)]) if self.n_frames else np.zeros((0, 4, 4))

    def set_poses(self, P):
        P = np.ascontiguousarray(P, dtype=np.float64)
        if P.shape != (self.n_frames, 4, 4):
            raise ValueError(f"expected ({self.n_frames}, 4, 4) poses")
        self._check(self.lib.pose_graph_set_poses(self.h, self.n_frames, P.ctypes.data_as(C.POINTER(C.c_double))))

    def optimize(self, check: bool = True) -> dict:
        s = L.pg_stats()
        rc = self.lib.pose_graph_optimize(self.h, C.byref(s))
        d = stats_to_dict(s, self.config.gn_iters)
        d["status"] = rc
        if check:
            self._check(rc)
        return d

    def linearize(self):
        N = self.n_frames
        H = np.zeros((6 * N, 6 * N))
        g = np.zeros(6 * N)
        s = L.pg_stats()
        self._check(self.lib.pose_graph_linearize(self.h, H.ctypes.data_as(C.POINTER(C.c_double)),
                                                  g.ctypes.data_as(C.POINTER(C.c_double)), C.byref(s)))
        return H, g, dict(energy_f=s.energy_f[0], energy_g=s.energy_g[0], n_valid_g=s.n_valid_g[0],
                          n_valid_f=s.n_valid_f[0], src_pixels=s.src_pixels)

    def associate(self, i: int, j: int):
        hw = self.camera.width * self.camera.height
        tgt = np.zeros(hw, np.int32)
        r = np.zeros(hw, np.float32)
        uv = np.zeros(2 * hw, np.float32)
        self._check(self.lib.pose_graph_associate(self.h, i, j, tgt.ctypes.data_as(C.POINTER(C.c_int32)),
                                                  r.ctypes.data_as(C.POINTER(C.c_float)),
                                                  uv.ctypes.data_as(C.POINTER(C.c_float))))
        return tgt, r, uv.reshape(hw, 2)

    def frame_info(self, i: int, with_map: bool = True):
        """(packed map (H, W, 4) or None, number of valid source pixels)."""
        n = C.c_int()
        if not with_map:
            self._check(self.lib.pose_graph_frame_info(self.h, i, None, C.byref(n)))
            return None, n.value
        hw = self.camera.width * self.camera.height
        m = np.zeros(4 * hw, np.float32)
        self._check(self.lib.pose_graph_frame_info(self.h, i, m.ctypes.data_as(C.POINTER(C.c_float)), C.byref(n)))
        return m.reshape(self.camera.height, self.camera.width, 4), n.value

    def set_mlp(self, params_fp16):
        """Network parameters of the learned weighting (1313 values, fp16)."""
        p = np.ascontiguousarray(params_fp16, dtype=np.float16)
        self._check(self.lib.pose_graph_set_mlp(self.h, C.c_void_p(p.ctypes.data), p.nbytes))

    def pair_features(self, i: int, j: int, iteration: int = 0, sigma: bool = False, out=None):
        """Learned-weighting features of ordered pair (i, j) at the current
        poses: (features (H*W, 6), sigma (H*W) or None, target (H*W)).  With
        out = (features, sigma, target) torch tensors on the device they are
        filled in place (sigma may be None) and returned."""
        hw = self.camera.width * self.camera.height
        if out is not None:
            f, sg, t = out
            self._check(self.lib.pose_graph_pair_features(
                self.h, i, j, iteration, C.c_void_p(f.data_ptr()),
                C.c_void_p(sg.data_ptr()) if sg is not None else None, C.c_void_p(t.data_ptr())))
            return f, sg, t
        f = np.zeros((hw, 6), np.float32)
        t = np.zeros(hw, np.int32)
        sg = np.zeros(hw, np.float32) if sigma else None
        self._check(self.lib.pose_graph_pair_features(self.h, i, j, iteration, C.c_void_p(f.ctypes.data),
                                                      C.c_void_p(sg.ctypes.data) if sigma else None,
                                                      C.c_void_p(t.ctypes.data)))
        return f, sg, t

    def time_assoc(self, reps: int = 100) -> float:
        """Milliseconds per association launch (reps back-to-back launches
        between HIP events on the graph's stream)."""
        ms = C.c_double()
        self._check(self.lib.pose_graph_time_assoc(self.h, int(reps), C.byref(ms)))
        return ms.value

    def ransac(self, pairs, uv_i, uv_j, samples, delta: float = 0.005, alpha: float = float(np.deg2rad(45.0)),
               install: bool = False, scores: bool = False):
        """Coarse registration by RANSAC of ordered node pairs (Sec. IV-B) on
        the GPU: uv_i / uv_j are lists (one (n_q, 2) array per pair),
        samples an (n_pairs, n_hyp, 3) array of match indices.  Returns
        dict(best (n_pairs,), T (n_pairs, 4, 4) frame-j camera -> frame-i
        camera, inliers (list of (n_q,) bools), and score (n_pairs, n_hyp)
        when asked); install=True makes the inliers the pairs' feature
        matches."""
        npairs = len(pairs)
        samples = np.ascontiguousarray(samples, np.int32).reshape(npairs, -1, 3)
        n_hyp = samples.shape[1]
        counts = [len(np.asarray(u).reshape(-1, 2)) for u in uv_i]
        off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(counts)]), np.int32)
        ui = np.ascontiguousarray(np.concatenate([np.asarray(u, np.float32).reshape(-1, 2) for u in uv_i]
                                                 + [np.zeros((1, 2), np.float32)]))
        uj = np.ascontiguousarray(np.concatenate([np.asarray(u, np.float32).reshape(-1, 2) for u in uv_j]
                                                 + [np.zeros((1, 2), np.float32)]))
        pi = np.ascontiguousarray([p[0] for p in pairs], np.int32)
        pj = np.ascontiguousarray([p[1] for p in pairs], np.int32)
        best = np.zeros(npairs, np.int32)
        T = np.zeros((npairs, 4, 4))
        inl = np.zeros(max(int(off[-1]), 1), np.uint8)
        sc = np.zeros((npairs, n_hyp), np.int32) if scores else None
        vp = lambda a: a.ctypes.data_as(C.c_void_p)
        self._check(self.lib.pose_graph_ransac(self.h, npairs, vp(pi), vp(pj), vp(off), vp(ui), vp(uj), n_hyp,
                                               vp(samples), float(delta), float(alpha), int(bool(install)),
                                               vp(best), vp(sc) if scores else None, vp(T), vp(inl)))
        out = dict(best=best, T=T, inliers=[inl[off[q]:off[q + 1]].astype(bool) for q in range(npairs)])
        if scores:
            out["score"] = sc
        return out

    def prune(self):
        """Pruning pass at the current poses: (score (N, H*W), keep (N, H*W))."""
        n = self.n_frames * self.camera.width * self.camera.height
        sc = np.zeros(n, np.float32)
        kp = np.zeros(n, np.uint8)
        self._check(self.lib.pose_graph_prune(self.h, C.c_void_p(sc.ctypes.data), C.c_void_p(kp.ctypes.data)))
        return sc.reshape(self.n_frames, -1), kp.reshape(self.n_frames, -1).astype(bool)


class MlpTrainer:
    """Trainer of the learned weighting network (pg_mlp_* handle).  Batches
    are device tensors: x (n, 6) float32, labels (n,) float32."""

    N_PARAMS = 1313

    def __init__(self, max_samples: int, stream=None):
        self.lib = L.load()
        st = _current_stream() if stream is None else C.c_void_p(stream if isinstance(stream, int)
                                                                else stream.cuda_stream)
        h = C.c_void_p()
        rc = self.lib.pg_mlp_create(int(max_samples), st, C.byref(h))
        if rc != L.PG_OK:
            raise PoseGraphError(rc, self.lib.pg_mlp_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc != L.PG_OK:
            raise PoseGraphError(rc, self.lib.pg_mlp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.pg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _dev(t, cols=None):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("expected a contiguous float32 device tensor")
        if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
            raise ValueError(f"expected shape (n, {cols})")
        return C.c_void_p(t.data_ptr())

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (self.N_PARAMS,):
            raise ValueError("expected 1313 parameters")
        self._check(self.lib.pg_mlp_set_params(self.h, C.c_void_p(p.ctypes.data)))

    def params(self):
        p = np.zeros(self.N_PARAMS, np.float32)
        self._check(self.lib.pg_mlp_get_params(self.h, C.c_void_p(p.ctypes.data), None))
        return p

    def params_fp16(self):
        p = np.zeros(self.N_PARAMS, np.float16)
        self._check(self.lib.pg_mlp_get_params(self.h, None, C.c_void_p(p.ctypes.data)))
        return p

    def loss_grad(self, x, labels):
        loss = C.c_double()
        g = np.zeros(self.N_PARAMS)
        self._check(self.lib.pg_mlp_loss_grad(self.h, self._dev(x, 6), self._dev(labels), x.shape[0],
                                              C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_double))))
        return loss.value, g

    def adam_step(self, x, labels, lr: float, want_loss: bool = False):
        loss = C.c_double()
        self._check(self.lib.pg_mlp_adam_step(self.h, self._dev(x, 6), self._dev(labels), x.shape[0], float(lr),
                                              C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def forward(self, x, y):
        self._check(self.lib.pg_mlp_forward(self.h, self._dev(x, 6), x.shape[0], self._dev(y)))
        return y


def optimize_batch(graphs: Sequence[PoseGraph], check: bool = True):
    lib = L.load()
    n = len(graphs)
    arr = (C.c_void_p * n)(*[g.h.value for g in graphs])
    stats = (L.pg_stats * n)()
    rc = lib.pose_graph_optimize_batch(arr, n, stats)
    if check and rc != L.PG_OK:
        msg = lib.pose_graph_last_error(graphs[0].h).decode()
        raise PoseGraphError(rc, msg)
    out = [stats_to_dict(stats[k], graphs[k].config.gn_iters) for k in range(n)]
    return rc, out


def from_synth(g, config: Optional[Config] = None, stream=None, device_inputs: bool = False) -> PoseGraph:
    """Fill a PoseGraph with a synthetic window (frames, poses, matches)."""
    cfg = config or Config(max_frames=max(g.n_frames, 2))
    pg = PoseGraph(Camera(g.width, g.height, g.fx, g.fy, g.cx, g.cy), cfg, stream)
    conv = (lambda a: a)
    if device_inputs:
        import torch
        conv = (lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda())
    for k in range(g.n_frames):
        pg.add_frame(conv(g.depth[k]), conv(g.mask[k]), g.poses_init[k], fixed=bool(g.fixed[k]))
    for m in g.matches:
        pg.add_matches(m.i, m.j, conv(m.uv_i), conv(m.uv_j))
    if device_inputs:
        import torch
        torch.cuda.synchronize()
    return pg
