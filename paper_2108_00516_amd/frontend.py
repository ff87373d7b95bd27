"""Python binding of the front-end entry points (include/pg_frontend.h):
keypoint descriptor matching on the GPU (Sec. IV-B).  Argument marshalling
only; torch supplies the device memory and the stream."""
from __future__ import annotations

import ctypes as C
from typing import Sequence, Tuple

import numpy as np

from . import _lib as L


class FrontendError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != L.PG_OK:
        msg = L.load().pg_frontend_last_error().decode()
        raise FrontendError(f"{what}: {L.STATUS_NAMES.get(rc, rc)}: {msg}")


def match_descriptors(desc, set_off: Sequence[int], pairs: Sequence[Tuple[int, int]], ratio: float = 1.0,
                      stream=None, with_distances: bool = True, noalloc: bool = False):
    """Mutual nearest-neighbour matching of descriptor sets on the GPU.

    desc: (rows, dim) float32 CUDA tensor; set s is rows set_off[s] ..
    set_off[s + 1] - 1.  pairs: (set a, set b) per pair.  Returns (match, d1,
    d2) CUDA tensors laid out pair after pair (na entries each; d1 / d2 None
    when with_distances is False).  noalloc selects the entry point whose
    scratch is the library's fixed array (no device allocation in the call)."""
    import torch
    lib = L.load()
    if not (desc.is_cuda and desc.dtype == torch.float32 and desc.dim() == 2 and desc.is_contiguous()):
        raise FrontendError("desc must be a contiguous (rows, dim) float32 CUDA tensor")
    off = np.ascontiguousarray(set_off, np.int32)
    pa = np.ascontiguousarray([p[0] for p in pairs], np.int32)
    pb = np.ascontiguousarray([p[1] for p in pairs], np.int32)
    n_out = int(sum(off[a + 1] - off[a] for a in pa)) if len(pa) else 0
    dev = desc.device
    match = torch.empty(max(n_out, 1), dtype=torch.int32, device=dev)
    d1 = torch.empty(max(n_out, 1), dtype=torch.float64, device=dev) if with_distances else None
    d2 = torch.empty(max(n_out, 1), dtype=torch.float64, device=dev) if with_distances else None
    st = (stream or torch.cuda.current_stream(dev)).cuda_stream
    fn = lib.pg_match_descriptors_noalloc if noalloc else lib.pg_match_descriptors
    rc = fn(
        C.c_void_p(desc.data_ptr()), off.ctypes.data_as(C.c_void_p), len(off) - 1, desc.shape[1],
        pa.ctypes.data_as(C.c_void_p), pb.ctypes.data_as(C.c_void_p), len(pa), float(ratio),
        C.c_void_p(match.data_ptr()), C.c_void_p(d1.data_ptr()) if d1 is not None else None,
        C.c_void_p(d2.data_ptr()) if d2 is not None else None, C.c_void_p(st))
    _check(rc, "pg_match_descriptors_noalloc" if noalloc else "pg_match_descriptors")
    return match[:n_out], (d1[:n_out] if d1 is not None else None), (d2[:n_out] if d2 is not None else None)


def select_keyframes(T_pool, T_cur, K: int = 15, novel_deg: float = 10.0, stream=None):
    """Greedy keyframe selection and novelty test of the memory pool
    (Sec. IV-C, IV-E) on the GPU.  T_pool: (n, 4, 4) poses (NumPy, or a CUDA
    float64 tensor); T_cur: (4, 4).  Returns (selected pool indices in
    selection order, novel flag, per-keyframe cost sums)."""
    lib = L.load()
    Tc = np.ascontiguousarray(T_cur, np.float64).reshape(16)
    if hasattr(T_pool, "data_ptr"):
        n = int(T_pool.shape[0])
        ptr = C.c_void_p(T_pool.data_ptr())
    else:
        Tp = np.ascontiguousarray(T_pool, np.float64).reshape(-1, 16)
        n = Tp.shape[0]
        ptr = Tp.ctypes.data_as(C.c_void_p)
    sel = np.zeros(max(K, 1), np.int32)
    nsel = C.c_int(0)
    novel = C.c_int(0)
    cost = np.zeros(max(n, 1))
    st = None
    if stream is not None:
        st = C.c_void_p(stream.cuda_stream)
    rc = lib.pg_select_keyframes(ptr, n, Tc.ctypes.data_as(C.c_void_p), int(K), float(np.deg2rad(novel_deg)),
                                 sel.ctypes.data_as(C.c_void_p), C.byref(nsel), C.byref(novel),
                                 cost.ctypes.data_as(C.c_void_p), st)
    _check(rc, "pg_select_keyframes")
    return sel[:nsel.value].copy(), bool(novel.value), cost[:n]
