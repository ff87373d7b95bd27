"""Shared helpers of the GPU parity tests (comparison rules only; no method
arithmetic)."""
import numpy as np

import oracle

# Tolerances (the stated parity bar): per pose 1e-5 rad / 1e-5 m; J^T W J
# within 1e-5 relative (Frobenius, whole matrix and each diagonal 6x6 block);
# each gradient entry within 1e-5 of the sum of magnitudes of its contributions.
POSE_TOL_RAD = 1e-5
POSE_TOL_M = 1e-5
H_REL_TOL = 1e-5
G_REL_TOL = 1e-5


def max_pose_diff(Pa, Pb):
    worst_r, worst_t = 0.0, 0.0
    for a, b in zip(Pa, Pb):
        r, t = oracle.pose_error(a, b)
        worst_r, worst_t = max(worst_r, r), max(worst_t, t)
    return worst_r, worst_t


def check_normal_equations(H_gpu, g_gpu, lin, tol_h=H_REL_TOL, tol_g=G_REL_TOL):
    H, g = lin["H"], lin["g"]
    rel = np.linalg.norm(H_gpu - H) / np.linalg.norm(H)
    assert rel <= tol_h, f"H relative Frobenius error {rel:.3e}"
    n = H.shape[0] // 6
    for k in range(n):
        blk = slice(6 * k, 6 * k + 6)
        nb = np.linalg.norm(H[blk, blk])
        if nb > 0:
            e = np.linalg.norm(H_gpu[blk, blk] - H[blk, blk]) / nb
            assert e <= tol_h, f"diagonal block {k}: {e:.3e}"
    scale = lin["g_abs"]
    err = np.abs(g_gpu - g)
    bad = err > tol_g * np.maximum(scale, 1e-30)
    assert not bad.any(), f"g entries off: {np.flatnonzero(bad)} err {err[bad]} scale {scale[bad]}"
    return rel


def near_half_integer(x, tol):
    return np.abs((x - np.floor(x)) - 0.5) <= tol
