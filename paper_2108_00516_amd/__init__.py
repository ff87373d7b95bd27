"""MI355X (gfx950) implementation of the online pose-graph optimisation of
BundleTrack (Wen & Bekris, IROS 2021), Sec. IV-D, behind the C ABI of
include/posegraph.h.  The HIP library must be built (build.py) before use."""
from .posegraph import (Camera, Config, MlpTrainer, PoseGraph, PoseGraphError, from_synth,  # noqa: F401
                        optimize_batch)
from . import _lib  # noqa: F401
