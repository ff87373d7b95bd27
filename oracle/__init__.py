"""FP64 CPU oracle of the pose-graph optimisation (Sec. IV-D, Eqs. 1-3 and the
Gauss-Newton step).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke
check and the CPU-baseline leg of the benchmark, never by the GPU library.

The numerics live in ``oracle.c`` (plain C, FP64); this module builds it with
gcc and marshals NumPy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OK, ERR_ARG, ERR_SINGULAR = 0, -1, -5
MAX_ITERS = 64


# A sanitized build (AddressSanitizer + UndefinedBehaviorSanitizer, every
# finding fatal) for the checker's own tests; ORACLE_LIB selects the library
# this module loads (the process must then preload the ASan runtime).
_SAN_SO = os.path.join(_HERE, "liboracle_san.so")


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP), or with
    sanitize=True into liboracle_san.so with -fsanitize=address,undefined."""
    so = _SAN_SO if sanitize else _SO
    if force or not os.path.exists(so):
        tmp = so + ".tmp"
        san = (["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
               if sanitize else [])
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               "-Wno-unused-parameter", *san, _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, so)
    return so


class Problem(C.Structure):
    _fields_ = [
        ("n_frames", C.c_int), ("width", C.c_int), ("height", C.c_int),
        ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
        ("depth", C.POINTER(C.c_float)), ("mask", C.POINTER(C.c_ubyte)), ("fixed", C.POINTER(C.c_int)),
        ("n_match_sets", C.c_int),
        ("match_i", C.POINTER(C.c_int)), ("match_j", C.POINTER(C.c_int)),
        ("match_n", C.POINTER(C.c_int)), ("match_off", C.POINTER(C.c_int)),
        ("uv_i", C.POINTER(C.c_float)), ("uv_j", C.POINTER(C.c_float)),
        ("lambda_f", C.c_double), ("lambda_g", C.c_double),
        ("huber_f", C.c_double), ("huber_g", C.c_double),
        ("gate_dist", C.c_double), ("gate_angle", C.c_double),
        ("mlp", C.POINTER(C.c_double)), ("keep", C.POINTER(C.c_ubyte)),
        ("prune_frac", C.c_double), ("mlp_iters", C.c_int), ("iteration", C.c_int),
    ]


class LinStats(C.Structure):
    _fields_ = [("energy_f", C.c_double), ("energy_g", C.c_double),
                ("n_valid_g", C.c_longlong), ("n_valid_f", C.c_longlong)]


class OptStats(C.Structure):
    _fields_ = [("iters_done", C.c_int),
                ("energy_f", C.c_double * MAX_ITERS), ("energy_g", C.c_double * MAX_ITERS),
                ("n_valid_g", C.c_longlong * MAX_ITERS), ("n_valid_f", C.c_longlong * MAX_ITERS)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB") or _SO
        if path == _SO and not os.path.exists(_SO):
            build()
        L = C.CDLL(path)
        P = C.POINTER
        dp = P(C.c_double)
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_rot_geodesic.restype = C.c_double
        L.orc_rot_geodesic.argtypes = [dp, dp]
        L.orc_select_keyframes.argtypes = [C.c_int, dp, dp, C.c_int, P(C.c_int), P(C.c_int), dp]
        L.orc_novel_view.argtypes = [C.c_int, dp, dp, C.c_double]
        L.orc_get_threads.restype = C.c_int
        L.orc_preprocess_frame.argtypes = [P(Problem), C.c_int, dp, dp, P(C.c_ubyte)]
        L.orc_linearize.argtypes = [P(Problem), dp, dp, dp, dp, dp, P(LinStats)]
        L.orc_optimize.argtypes = [P(Problem), dp, C.c_int, P(OptStats)]
        L.orc_linearize_given.argtypes = [P(Problem), dp, P(C.c_int), dp, dp, dp, dp, P(LinStats)]
        L.orc_associate.argtypes = [P(Problem), dp, C.c_int, C.c_int, P(C.c_int), dp, dp, dp]
        L.orc_dense_frozen.argtypes = [P(Problem), dp, C.c_int, C.c_int, C.c_int, P(C.c_int), P(C.c_int), dp, dp]
        L.orc_feature_eval.argtypes = [P(Problem), dp, C.c_int, C.c_int, dp, dp]
        L.orc_se3_exp.argtypes = [dp, dp]
        L.orc_huber_rho.argtypes = [C.c_double, C.c_double]
        L.orc_huber_rho.restype = C.c_double
        L.orc_huber_weight.argtypes = [C.c_double, C.c_double]
        L.orc_huber_weight.restype = C.c_double
        L.orc_cholesky_solve.argtypes = [C.c_int, dp, dp, dp]
        L.orc_mlp_forward.argtypes = [dp, C.c_int, dp, dp]
        L.orc_mlp_forward_half.argtypes = [dp, C.c_int, dp, dp]
        L.orc_mlp_trace_half.argtypes = [dp, C.c_int, dp, dp, dp, dp]
        L.orc_round_half.argtypes = [C.c_double]
        L.orc_round_half.restype = C.c_double
        L.orc_pair_features.argtypes = [P(Problem), dp, C.c_int, C.c_int, C.c_int, P(C.c_int), dp]
        L.orc_pairs_features.argtypes = [P(Problem), dp, C.c_int, P(C.c_int), P(C.c_int), C.c_int, P(C.c_int), dp]
        L.orc_prune_scores.argtypes = [P(Problem), dp, dp]
        L.orc_prune_select.argtypes = [P(Problem), dp, C.c_double, P(C.c_ubyte)]
        L.orc_arun.argtypes = [C.c_int, dp, dp, dp]
        L.orc_ransac_score.restype = C.c_int
        L.orc_ransac_score.argtypes = [C.c_int, dp, dp, dp, dp, P(C.c_ubyte), P(C.c_int), C.c_double, C.c_double,
                                       dp, P(C.c_ubyte)]
        L.orc_ransac_pairs.argtypes = [P(Problem), C.c_int, P(C.c_int), P(C.c_int), P(C.c_int), P(C.c_float),
                                       P(C.c_float), C.c_int, P(C.c_int), C.c_double, C.c_double, P(C.c_int),
                                       P(C.c_int), dp, P(C.c_ubyte)]
        L.orc_match_descriptors.argtypes = [C.c_int, P(C.c_float), C.c_int, P(C.c_float), C.c_int, C.c_double,
                                            P(C.c_int), dp, dp]
        L.orc_mlp_bce.argtypes = [dp, C.c_int, dp, dp, dp]
        L.orc_mlp_bce.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


@dataclass
class Params:
    """The method's constants (readings of Sec. IV-B/IV-D, see the design notes):
    lambda_1 = lambda_2 = 1 (Eq. 1 weights as used in the paper's experiments);
    Huber thresholds 5 mm (the paper's inlier distance scale, RANSAC delta);
    dense gates 1 cm / 30 degrees."""
    lambda_f: float = 1.0
    lambda_g: float = 1.0
    huber_f: float = 0.005
    huber_g: float = 0.005
    gate_dist: float = 0.01
    gate_angle: float = float(np.deg2rad(30.0))
    mlp: Optional[np.ndarray] = None      # 1313 network parameters (learned weighting)
    prune_frac: float = 0.0               # fraction of source pixels pruned by optimize
    mlp_iters: int = 7                    # iteration-feature normalisation


class OracleProblem:
    """Owns the contiguous arrays an orc_problem borrows."""

    def __init__(self, depth, mask, fx, fy, cx, cy, fixed=None, matches: Sequence = (),
                 params: Optional[Params] = None):
        self.depth = np.ascontiguousarray(depth, dtype=np.float32)
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        N, H, W = self.depth.shape
        self.fixed = np.ascontiguousarray(
            np.zeros(N, np.int32) if fixed is None else np.asarray(fixed, np.int32))
        self.params = params or Params()
        mi, mj, mn, mo, ui, uj = [], [], [], [], [], []
        off = 0
        for m in matches:
            a, b = np.asarray(m.uv_i, np.float32).reshape(-1, 2), np.asarray(m.uv_j, np.float32).reshape(-1, 2)
            mi.append(m.i), mj.append(m.j), mn.append(len(a)), mo.append(off)
            ui.append(a), uj.append(b)
            off += len(a)
        self.match_i = np.asarray(mi, np.int32)
        self.match_j = np.asarray(mj, np.int32)
        self.match_n = np.asarray(mn, np.int32)
        self.match_off = np.asarray(mo, np.int32)
        self.uv_i = np.ascontiguousarray(np.concatenate(ui) if ui else np.zeros((1, 2), np.float32))
        self.uv_j = np.ascontiguousarray(np.concatenate(uj) if uj else np.zeros((1, 2), np.float32))
        self.n_frames, self.height, self.width = N, H, W
        self.fx, self.fy, self.cx, self.cy = float(fx), float(fy), float(cx), float(cy)
        self.c = Problem()
        self._fill()

    def _fill(self):
        c, p = self.c, self.params
        c.n_frames, c.width, c.height = self.n_frames, self.width, self.height
        c.fx, c.fy, c.cx, c.cy = self.fx, self.fy, self.cx, self.cy
        c.depth = _ptr(self.depth, C.c_float)
        c.mask = _ptr(self.mask, C.c_ubyte)
        c.fixed = _ptr(self.fixed, C.c_int)
        c.n_match_sets = len(self.match_i)
        c.match_i = _ptr(self.match_i, C.c_int) if len(self.match_i) else None
        c.match_j = _ptr(self.match_j, C.c_int) if len(self.match_j) else None
        c.match_n = _ptr(self.match_n, C.c_int) if len(self.match_n) else None
        c.match_off = _ptr(self.match_off, C.c_int) if len(self.match_off) else None
        c.uv_i = _ptr(self.uv_i, C.c_float)
        c.uv_j = _ptr(self.uv_j, C.c_float)
        c.lambda_f, c.lambda_g = p.lambda_f, p.lambda_g
        c.huber_f, c.huber_g = p.huber_f, p.huber_g
        c.gate_dist, c.gate_angle = p.gate_dist, p.gate_angle
        self._mlp = None if p.mlp is None else np.ascontiguousarray(p.mlp, np.float64)
        c.mlp = _ptr(self._mlp, C.c_double) if self._mlp is not None else None
        c.keep = _ptr(self._keep, C.c_ubyte) if getattr(self, "_keep", None) is not None else None
        c.prune_frac = p.prune_frac
        c.mlp_iters = p.mlp_iters
        c.iteration = getattr(self, "_iteration", 0)

    def set_keep(self, keep):
        """Kept source pixels (n_frames, H, W) bytes, or None for all."""
        self._keep = None if keep is None else np.ascontiguousarray(keep, np.uint8).reshape(-1)
        self._fill()

    def set_iteration(self, it: int):
        self._iteration = int(it)
        self._fill()

    def pair_features(self, poses, i, j, iteration=0):
        poses = np.ascontiguousarray(poses, np.float64)
        hw = self.width * self.height
        tgt = np.zeros(hw, np.int32)
        f = np.zeros((hw, 6))
        rc = lib().orc_pair_features(C.byref(self.c), _ptr(poses, C.c_double), i, j, iteration,
                                     _ptr(tgt, C.c_int), _ptr(f, C.c_double))
        assert rc == OK
        return tgt, f

    def pairs_features(self, poses, pairs, iteration=0):
        """(targets (n, H*W), features (n, H*W, 6)) of the ordered pairs."""
        poses = np.ascontiguousarray(poses, np.float64)
        hw = self.width * self.height
        pi = np.ascontiguousarray([p[0] for p in pairs], np.int32)
        pj = np.ascontiguousarray([p[1] for p in pairs], np.int32)
        tgt = np.zeros((len(pairs), hw), np.int32)
        f = np.zeros((len(pairs), hw, 6))
        rc = lib().orc_pairs_features(C.byref(self.c), _ptr(poses, C.c_double), len(pairs), _ptr(pi, C.c_int),
                                      _ptr(pj, C.c_int), iteration, _ptr(tgt, C.c_int), _ptr(f, C.c_double))
        assert rc == OK
        return tgt, f

    def ransac(self, pairs, uv_i, uv_j, samples, delta=0.005, alpha=float(np.deg2rad(45.0)), scores=False):
        """RANSAC registration of each ordered pair (i, j) in pairs from its
        matches: uv_i / uv_j are lists (one (n_q, 2) array per pair), samples an
        (n_pairs, n_hyp, 3) array of match indices.  Returns dict(best (n_pairs,),
        T (n_pairs, 4, 4) frame-j camera -> frame-i camera, inliers (list of
        (n_q,) bools), and score (n_pairs, n_hyp) when asked)."""
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
        rc = lib().orc_ransac_pairs(C.byref(self.c), npairs, _ptr(pi, C.c_int), _ptr(pj, C.c_int),
                                    _ptr(off, C.c_int), _ptr(ui, C.c_float), _ptr(uj, C.c_float), n_hyp,
                                    _ptr(samples, C.c_int), float(delta), float(alpha), _ptr(best, C.c_int),
                                    _ptr(sc, C.c_int) if scores else None, _ptr(T, C.c_double),
                                    _ptr(inl, C.c_ubyte))
        assert rc == OK
        out = dict(best=best, T=T, inliers=[inl[off[q]:off[q + 1]].astype(bool) for q in range(npairs)])
        if scores:
            out["score"] = sc
        return out

    def prune_scores(self, poses):
        poses = np.ascontiguousarray(poses, np.float64)
        sc = np.zeros(self.n_frames * self.width * self.height)
        rc = lib().orc_prune_scores(C.byref(self.c), _ptr(poses, C.c_double), _ptr(sc, C.c_double))
        assert rc == OK
        return sc.reshape(self.n_frames, self.height, self.width)

    def prune_select(self, score, frac):
        sc = np.ascontiguousarray(score, np.float64)
        keep = np.zeros(sc.size, np.uint8)
        rc = lib().orc_prune_select(C.byref(self.c), _ptr(sc, C.c_double), float(frac), _ptr(keep, C.c_ubyte))
        assert rc == OK
        return keep.reshape(self.n_frames, self.height, self.width)

    def set_params(self, **kw):
        for k, v in kw.items():
            setattr(self.params, k, v)
        self._fill()

    @classmethod
    def from_synth(cls, g, params: Optional[Params] = None, clean: bool = False, matches=True):
        return cls(g.depth_clean if clean else g.depth, g.mask, g.fx, g.fy, g.cx, g.cy, g.fixed,
                   g.matches if matches else (), params)

    # ---------------------------------------------------------- entry points
    def preprocess(self, f):
        hw = self.width * self.height
        V = np.zeros(3 * hw)
        Nn = np.zeros(3 * hw)
        code = np.zeros(hw, np.uint8)
        rc = lib().orc_preprocess_frame(C.byref(self.c), f, _ptr(V, C.c_double), _ptr(Nn, C.c_double),
                                        _ptr(code, C.c_ubyte))
        assert rc == OK
        return (V.reshape(self.height, self.width, 3), Nn.reshape(self.height, self.width, 3),
                code.reshape(self.height, self.width))

    def linearize(self, poses):
        poses = np.ascontiguousarray(poses, np.float64)
        n6 = 6 * self.n_frames
        H = np.zeros((n6, n6))
        g = np.zeros(n6)
        Ha = np.zeros((n6, n6))
        ga = np.zeros(n6)
        st = LinStats()
        rc = lib().orc_linearize(C.byref(self.c), _ptr(poses, C.c_double), _ptr(H, C.c_double), _ptr(g, C.c_double),
                                 _ptr(Ha, C.c_double), _ptr(ga, C.c_double), C.byref(st))
        assert rc == OK, rc
        return dict(H=H, g=g, H_abs=Ha, g_abs=ga, energy_f=st.energy_f, energy_g=st.energy_g,
                    n_valid_g=st.n_valid_g, n_valid_f=st.n_valid_f)

    def linearize_given(self, poses, targets):
        """Normal equations with the dense association decisions given:
        targets is (N(N-1), H*W) int32, ordered pairs in lexicographic order."""
        poses = np.ascontiguousarray(poses, np.float64)
        tg = np.ascontiguousarray(targets, np.int32)
        N = self.n_frames
        assert tg.shape == (N * (N - 1), self.width * self.height)
        n6 = 6 * N
        H = np.zeros((n6, n6))
        g = np.zeros(n6)
        Ha = np.zeros((n6, n6))
        ga = np.zeros(n6)
        st = LinStats()
        rc = lib().orc_linearize_given(C.byref(self.c), _ptr(poses, C.c_double), _ptr(tg, C.c_int),
                                       _ptr(H, C.c_double), _ptr(g, C.c_double), _ptr(Ha, C.c_double),
                                       _ptr(ga, C.c_double), C.byref(st))
        assert rc == OK, rc
        return dict(H=H, g=g, H_abs=Ha, g_abs=ga, energy_f=st.energy_f, energy_g=st.energy_g,
                    n_valid_g=st.n_valid_g, n_valid_f=st.n_valid_f)

    def ordered_pairs(self):
        N = self.n_frames
        return [(i, j) for i in range(N) for j in range(N) if j != i]

    def optimize(self, poses, iters=7):
        P = np.ascontiguousarray(np.array(poses, np.float64, copy=True))
        st = OptStats()
        rc = lib().orc_optimize(C.byref(self.c), _ptr(P, C.c_double), int(iters), C.byref(st))
        k = st.iters_done
        return P, dict(status=rc, iters_done=k, energy_f=np.array(st.energy_f[:iters]),
                       energy_g=np.array(st.energy_g[:iters]), n_valid_g=np.array(st.n_valid_g[:iters]),
                       n_valid_f=np.array(st.n_valid_f[:iters]))

    def associate(self, poses, i, j):
        poses = np.ascontiguousarray(poses, np.float64)
        hw = self.width * self.height
        tgt = np.zeros(hw, np.int32)
        r = np.zeros(hw)
        proj = np.zeros(2 * hw)
        gate = np.zeros(2 * hw)
        rc = lib().orc_associate(C.byref(self.c), _ptr(poses, C.c_double), i, j, _ptr(tgt, C.c_int),
                                 _ptr(r, C.c_double), _ptr(proj, C.c_double), _ptr(gate, C.c_double))
        assert rc == OK
        return tgt, r, proj.reshape(hw, 2), gate.reshape(hw, 2)

    def dense_frozen(self, poses, i, j, src, tgt):
        poses = np.ascontiguousarray(poses, np.float64)
        src = np.ascontiguousarray(src, np.int32)
        tgt = np.ascontiguousarray(tgt, np.int32)
        n = len(src)
        r = np.zeros(n)
        J = np.zeros((n, 12))
        rc = lib().orc_dense_frozen(C.byref(self.c), _ptr(poses, C.c_double), i, j, n, _ptr(src, C.c_int),
                                    _ptr(tgt, C.c_int), _ptr(r, C.c_double), _ptr(J, C.c_double))
        assert rc == OK
        return r, J

    def feature_eval(self, poses, s, k):
        poses = np.ascontiguousarray(poses, np.float64)
        e = np.zeros(3)
        J = np.zeros((3, 12))
        ok = lib().orc_feature_eval(C.byref(self.c), _ptr(poses, C.c_double), s, k, _ptr(e, C.c_double),
                                    _ptr(J, C.c_double))
        return bool(ok), e, J


def se3_exp(xi) -> np.ndarray:
    xi = np.ascontiguousarray(xi, np.float64)
    T = np.zeros(16)
    lib().orc_se3_exp(_ptr(xi, C.c_double), _ptr(T, C.c_double))
    return T.reshape(4, 4)


def huber_rho(s, delta):
    return lib().orc_huber_rho(float(s), float(delta))


def huber_weight(s, delta):
    return lib().orc_huber_weight(float(s), float(delta))


def cholesky_solve(A, b):
    A = np.ascontiguousarray(A, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros_like(b)
    rc = lib().orc_cholesky_solve(len(b), _ptr(A, C.c_double), _ptr(b, C.c_double), _ptr(x, C.c_double))
    return rc, x


MLP_PARAMS = 1313


def mlp_forward(params, x):
    """Outputs (n,) of the 6-32-32-1 weighting network for inputs (n, 6)."""
    p = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 6)
    y = np.zeros(len(x))
    lib().orc_mlp_forward(_ptr(p, C.c_double), len(x), _ptr(x, C.c_double), _ptr(y, C.c_double))
    return y


def mlp_forward_half(params, x):
    """Outputs of the network as the dense term evaluates it, "in FP16":
    binary16 parameters, every layer's input (features, both hidden layers'
    activations) rounded to binary16, exact products and sums."""
    p = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 6)
    y = np.zeros(len(x))
    lib().orc_mlp_forward_half(_ptr(p, C.c_double), len(x), _ptr(x, C.c_double), _ptr(y, C.c_double))
    return y


def mlp_trace_half(params, x):
    """(s1, s2, z) of the FP16 evaluation: the exact pre-activations (n, 32)
    of the two hidden layers, each from its layer's binary16 inputs, and the
    logits (n,)."""
    p = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 6)
    s1 = np.zeros((len(x), 32))
    s2 = np.zeros((len(x), 32))
    z = np.zeros(len(x))
    lib().orc_mlp_trace_half(_ptr(p, C.c_double), len(x), _ptr(x, C.c_double), _ptr(s1, C.c_double),
                             _ptr(s2, C.c_double), _ptr(z, C.c_double))
    return s1, s2, z


def arun(a, b):
    """(rc, T): least-squares rigid transform with R b + t ~ a for (k, 3)
    point arrays (Arun et al.)."""
    a = np.ascontiguousarray(a, np.float64).reshape(-1, 3)
    b = np.ascontiguousarray(b, np.float64).reshape(-1, 3)
    T = np.zeros((4, 4))
    rc = lib().orc_arun(len(a), _ptr(a, C.c_double), _ptr(b, C.c_double), _ptr(T, C.c_double))
    return rc, T


def ransac_score(a, na, b, nb, valid, sample, delta=0.005, alpha=float(np.deg2rad(45.0))):
    """(score, T, inlier flags) of one hypothesis on explicit geometry."""
    arrs = [np.ascontiguousarray(v, np.float64).reshape(-1, 3) for v in (a, na, b, nb)]
    n = len(arrs[0])
    valid = np.ascontiguousarray(valid, np.uint8)
    smp = np.ascontiguousarray(sample, np.int32)
    T = np.zeros((4, 4))
    inl = np.zeros(max(n, 1), np.uint8)
    s = lib().orc_ransac_score(n, *[_ptr(v, C.c_double) for v in arrs], _ptr(valid, C.c_ubyte), _ptr(smp, C.c_int),
                               float(delta), float(alpha), _ptr(T, C.c_double), _ptr(inl, C.c_ubyte))
    return s, T, inl[:n].astype(bool)


def match_descriptors(A, B, ratio=1.0):
    """(match (na,), d1 (na,), d2 (na,)): mutual nearest neighbours of the
    FP32 descriptor rows of A in B (squared Euclidean distances, FP64), with
    the ratio test when ratio < 1."""
    A = np.ascontiguousarray(A, np.float32)
    B = np.ascontiguousarray(B, np.float32)
    na, nb = len(A), len(B)
    dim = A.shape[1] if A.ndim == 2 else B.shape[1]
    m = np.zeros(max(na, 1), np.int32)
    d1 = np.zeros(max(na, 1))
    d2 = np.zeros(max(na, 1))
    rc = lib().orc_match_descriptors(na, _ptr(A, C.c_float), nb, _ptr(B, C.c_float), int(dim), float(ratio),
                                     _ptr(m, C.c_int), _ptr(d1, C.c_double), _ptr(d2, C.c_double))
    assert rc == OK
    return m[:na], d1[:na], d2[:na]


def round_half(x):
    return lib().orc_round_half(float(x))


def mlp_bce(params, x, labels, with_grad=True):
    """(mean binary cross-entropy, gradient (1313,) or None)."""
    p = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 6)
    t = np.ascontiguousarray(labels, np.float64)
    g = np.zeros(MLP_PARAMS) if with_grad else None
    loss = lib().orc_mlp_bce(_ptr(p, C.c_double), len(x), _ptr(x, C.c_double), _ptr(t, C.c_double),
                             _ptr(g, C.c_double) if with_grad else None)
    return loss, g


def rot_geodesic(Ta, Tb) -> float:
    a = np.ascontiguousarray(Ta, np.float64).reshape(16)
    b = np.ascontiguousarray(Tb, np.float64).reshape(16)
    return float(lib().orc_rot_geodesic(_ptr(a, C.c_double), _ptr(b, C.c_double)))


def select_keyframes(T_pool, T_cur, K):
    """Greedy keyframe selection (Sec. IV-C): (selected indices in selection
    order, final cost sums)."""
    P = np.ascontiguousarray(T_pool, np.float64).reshape(-1, 16)
    t = np.ascontiguousarray(T_cur, np.float64).reshape(16)
    sel = np.zeros(max(K, 1), np.int32)
    nsel = C.c_int(0)
    cost = np.zeros(len(P))
    rc = lib().orc_select_keyframes(len(P), _ptr(P, C.c_double), _ptr(t, C.c_double), int(K),
                                    _ptr(sel, C.c_int), C.byref(nsel), _ptr(cost, C.c_double))
    assert rc == OK
    return sel[:nsel.value].copy(), cost


def novel_view(T_pool, T_cur, thresh=float(np.deg2rad(10.0))) -> bool:
    P = np.ascontiguousarray(T_pool, np.float64).reshape(-1, 16)
    t = np.ascontiguousarray(T_cur, np.float64).reshape(16)
    return bool(lib().orc_novel_view(len(P), _ptr(P, C.c_double), _ptr(t, C.c_double), float(thresh)))


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def pose_error(Ta, Tb):
    """(rotation angle in rad, translation distance in m) between two poses;
    the angle from atan2 of the skew and trace parts (accurate near zero)."""
    Ra, Rb = np.asarray(Ta)[:3, :3], np.asarray(Tb)[:3, :3]
    M = Ra @ Rb.T
    sk = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    ang = np.arctan2(np.linalg.norm(sk) / 2.0, (np.trace(M) - 1.0) / 2.0)
    return float(ang), float(np.linalg.norm(np.asarray(Ta)[:3, 3] - np.asarray(Tb)[:3, 3]))
