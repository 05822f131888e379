"""Quality metrics of the oracle (paper Sec. 7.1).

Test infrastructure: FP64, plain NumPy.

Misorientation between two cubic orientations is the smallest rotation angle
of R_a^T R_b S over the 24 proper rotations S of the cube.  A grain counts as
recovered when an estimated grain lies within the angle and position
thresholds (reading: 0.25 deg and 0.5 mm; the paper states no thresholds);
estimates are matched one-to-one, greedily by misorientation.
"""
from __future__ import annotations

import numpy as np

from . import crystal

_SYM = crystal.cubic_group()


def rotation_angle(R):
    c = (np.trace(R, axis1=-2, axis2=-1) - 1.0) / 2.0
    return np.arccos(np.clip(c, -1.0, 1.0))


def misorientation(qa, qb):
    """Radians, reduced over the cubic group; qa, qb [..,4]."""
    Ra = crystal.quat_to_R(qa)
    Rb = crystal.quat_to_R(qb)
    M = np.einsum("...ba,...bc->...ac", Ra, Rb)          # Ra^T Rb
    ang = rotation_angle(np.einsum("...ab,sbc->...sac", M, _SYM))
    return np.min(ang, axis=-1)


def match_grains(q_est, x_est, q_true, x_true, ang_tol_deg=0.25, pos_tol_mm=0.5):
    """Greedy one-to-one matching; returns (n_recovered, per-true matched index or -1)."""
    if len(q_est) == 0:
        return 0, -np.ones(len(q_true), dtype=np.int64)
    mis = np.degrees(misorientation(q_true[:, None, :], q_est[None, :, :]))
    dist = np.linalg.norm(x_true[:, None, :] - x_est[None, :, :], axis=-1)
    ok = (mis <= ang_tol_deg) & (dist <= pos_tol_mm)
    order = np.argsort(np.where(ok, mis, np.inf), axis=None)
    used_t, used_e = set(), set()
    match = -np.ones(len(q_true), dtype=np.int64)
    for flat in order:
        t, e = divmod(int(flat), len(q_est))
        if not ok[t, e]:
            break
        if t in used_t or e in used_e:
            continue
        used_t.add(t)
        used_e.add(e)
        match[t] = e
    return len(used_t), match
