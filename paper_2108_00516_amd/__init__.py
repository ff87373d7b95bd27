"""MI355X (gfx950) implementation of the online pose-graph optimisation of
BundleTrack (Wen & Bekris, IROS 2021), Sec. IV-D, behind the C ABI of
include/posegraph.h.  The HIP library must be built (build.py) before use."""
from .posegraph import Camera, Config, PoseGraph, PoseGraphError, from_synth, optimize_batch  # noqa: F401
from . import _lib  # noqa: F401
