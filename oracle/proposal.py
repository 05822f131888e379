"""Oracle of the learned proposal's inputs and outputs besides the network:
cheap-support features, training labels and top-fraction selection.

Test infrastructure: FP64, plain NumPy, brute force (no spatial index).

The paper seeds single-grain fitting with every start (Sec. 6.1) and
mentions learned indexers only as prior art (Sec. 2).  The learned proposal
ranks spot-pair candidates with a small network and keeps a top fraction for
the single-grain refinement; these definitions fix what its features and
labels are so that the GPU path can be checked.

Cheap support of a candidate (orientation R, position hypothesis x = 0, pair
drawn at rotation t):
  * the probe rotations are t_k = (t + floor(k T / 3)) mod T for k = 1, 2,
    away from the pair's own rotation;
  * the probe planes are the first n_support planes of the list (lowest
    order first) that have no parallel plane of lower order;
  * a probe plane is predicted at t_k on detector d by the forward model of
    Sec. 3.3 (lambda in band, tau > 0, strictly inside the detector);
  * it is hit when a detected spot of block (t_k, d) lies within `radius` mm
    of the prediction (detector-plane distance, <=);
  * feature 14 + (k - 1) = hits / max(predictions, 1).

Label of a candidate: 1 when both spots of its pair come from the same true
grain g and its orientation is within max_deg of g's, up to the 24 proper
cubic rotations; else 0.

Top-fraction selection: the k = ceil(frac * n) highest scores, equal scores
taken in increasing index order; the chosen indices are returned ascending.

Same-grain training pairs: pair k draws Philox4x32-10 counter (k, 0, 0, 7);
a = x0 mod n_obs; when spot a is an outlier or alone in its rotation among
its grain's spots the pair is (-1, -1), else b is the (x1 mod count)-th other
spot of that grain and rotation in index order.
"""
from __future__ import annotations

import math

import numpy as np

from . import crystal, metrics, philox

STREAM_SAME_PAIR = 7

E = np.array([1.0, 0.0, 0.0])


def probe_rotations(t, n_rot):
    return [(t + (k * n_rot) // 3) % n_rot for k in (1, 2)]


def probe_planes(planes, n_support):
    """Indices of the first n_support planes without a lower-order parallel plane."""
    m = np.arange(min(int(n_support), len(planes["d"])))
    return m[np.asarray(planes["harmonic_prev"])[m] < 0]


def predict(planes, geom, R, t, mset):
    """Predicted detector-local positions of planes mset at rotation t for a grain
    (R, x = 0): list of (det, s12 [2], margin), margin = distance of the
    visibility decision from its thresholds (band, tau, detector edge)."""
    out = []
    G = geom.G[t]
    for m in mset:
        u = G @ R @ planes["w"][m]
        lam = 2.0 * planes["d"][m] * u[0]
        if not (geom.lam_min <= lam <= geom.lam_max):
            continue
        mlam = min(abs(lam - geom.lam_min), abs(lam - geom.lam_max))
        r = E - 2.0 * u[0] * u
        for d in range(geom.n_det):
            nu, gam = geom.det_normal[d], geom.det_center[d]
            den = r @ nu
            if den == 0.0:
                continue
            tau = (gam @ nu) / den
            if not tau > 0.0:
                continue
            s12 = geom.to_local(d, tau * r)
            inf = np.max(np.abs(s12))
            if not inf < geom.det_half[d]:
                continue
            out.append((d, s12, min(mlam, abs(inf - geom.det_half[d]))))
    return out


def support(planes, geom, p12, offsets, q, t_pair, radius, n_support):
    """Cheap-support fractions [n, 2] of candidates q [n, 4] with pair rotations
    t_pair [n], and per candidate the number of decisions within 1e-6 of a
    threshold (band or detector edge in its own unit, hit distance in mm)."""
    q = np.atleast_2d(q)
    mset = probe_planes(planes, n_support)
    frac = np.zeros((len(q), 2))
    border = np.zeros(len(q), dtype=np.int64)
    for c in range(len(q)):
        R = crystal.quat_to_R(q[c])
        for k, t in enumerate(probe_rotations(int(t_pair[c]), geom.n_rot)):
            pred = predict(planes, geom, R, t, mset)
            hits = 0
            for d, s12, margin in pred:
                b = t * geom.n_det + d
                pts = p12[offsets[b]:offsets[b + 1]]
                dist = np.sqrt(np.sum((pts - s12) ** 2, axis=1)) if len(pts) else np.zeros(0)
                hits += bool(np.any(dist <= radius))
                border[c] += (margin < 1e-6) + int(np.any(np.abs(dist - radius) < 1e-6))
            frac[c, k] = hits / max(len(pred), 1)
    return frac, border


def labels(q, spot_a, spot_b, spot_grain, q_true, max_deg=2.0):
    """Training labels (0/1) and the misorientation (deg) to the pair's grain (inf
    when the two spots are not from one true grain)."""
    q = np.atleast_2d(q)
    ga = np.asarray(spot_grain)[np.asarray(spot_a)]
    gb = np.asarray(spot_grain)[np.asarray(spot_b)]
    same = (ga == gb) & (ga >= 0)
    mis = np.full(len(q), np.inf)
    if same.any():
        mis[same] = np.degrees(metrics.misorientation(q[same], np.atleast_2d(q_true)[ga[same]]))
    return (mis <= max_deg).astype(np.float64), mis


def labels_nearest(q, q_true, max_deg=1.0):
    """Training labels by the nearest true grain: 1 when the candidate
    orientation is within max_deg of some true grain (cubic symmetry), with the
    smallest misorientation (deg) and that grain (lowest index on ties; -1 and
    inf without true grains)."""
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    qt = np.atleast_2d(np.asarray(q_true, dtype=np.float64))
    if qt.shape[0] == 0 or qt.shape[1] == 0:
        return np.zeros(len(q)), np.full(len(q), np.inf), -np.ones(len(q), dtype=np.int64)
    mis = np.degrees(metrics.misorientation(q[:, None, :], qt[None, :, :]))
    near = np.argmin(mis, axis=1)
    m = mis[np.arange(len(q)), near]
    return (m <= max_deg).astype(np.float64), m, near


def select_top(score, frac):
    """Indices (ascending) of the ceil(frac * n) highest scores; ties by index."""
    score = np.asarray(score)
    n = len(score)
    k = min(n, int(math.ceil(frac * n)))
    order = sorted(range(n), key=lambda i: (-score[i], i))
    return np.sort(np.array(order[:k], dtype=np.int64))


def same_grain_pairs(offsets, spot_grain, n_det, n_pairs, seed):
    offsets = np.asarray(offsets)
    grain = np.asarray(spot_grain)
    n_obs = int(offsets[-1])
    k = np.arange(n_pairs)
    x0, x1, _, _ = philox.philox4x32_10(k, 0, 0, STREAM_SAME_PAIR, *philox.seed_key(seed))
    a_out = -np.ones(n_pairs, dtype=np.int64)
    b_out = -np.ones(n_pairs, dtype=np.int64)
    if n_obs == 0:
        return a_out, b_out
    for j in range(n_pairs):
        a = int(x0[j] % np.uint64(n_obs))
        if grain[a] < 0:
            continue
        blk = int(np.searchsorted(offsets, a, side="right") - 1)
        t = blk // n_det
        lo, hi = offsets[t * n_det], offsets[(t + 1) * n_det]
        mates = [i for i in range(lo, hi) if i != a and grain[i] == grain[a]]
        if not mates:
            continue
        a_out[j] = a
        b_out[j] = mates[int(x1[j] % np.uint64(len(mates)))]
    return a_out, b_out
