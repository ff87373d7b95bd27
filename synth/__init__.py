"""Seeded synthetic inputs (scene synthesis only; none of the method's arithmetic)."""
from .scene import PRESETS, SynthGraph, MatchSet, make_graph, render, perturb_pose, plane_frames, ransac_samples, make_keypoints, KeypointFrame  # noqa: F401
