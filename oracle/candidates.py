"""Spot-pair candidate orientations for the oracle.

Test infrastructure: FP64, plain NumPy.

The paper seeds single-grain fitting from a Sobol grid (Sec. 6.1).  The
candidates here come from pairs of detected spots instead: each spot of a
pair is read as a reflection of a grain at the sample centre (x = 0).
  * The unit vector from the centre to the spot is the diffracted ray rhat.
  * Inverting Eq. ray_mnt gives the lab plane normal u = (e - rhat)/|e - rhat|
    (u.e > 0), and sin(theta) = u.e = |e - rhat| / 2 (Eq. bragg).
  * The sample-frame normal is n = Gamma_t^T u.
  * A plane m can have produced the spot when 2 d_m sin(theta) lies in the band
    (Eq. wavelength_lambda).
For a pair (a, b) of the same rotation:
  * m_a runs over one representative per orbit of the 24 proper cubic
    rotations (the first plane of the orbit in list order; general families
    such as {321} split into two orbits) with its wavelength in band.
  * m_b runs over every plane in band that is not parallel to m_a.
  * A hypothesis is kept when the angle between w_a and w_b is within delta of
    the angle between n_a and n_b.
  * Its orientation solves Wahba's problem (App. A, Alg. Wahba) for the pairs
    (n_a, w_a), (n_b, w_b) and (n_a x n_b, w_a x w_b), the crossed vectors
    normalised, unit weights.
Pairs are drawn with Philox4x32-10 (counter (k, 0, 0, 5)):
  * word 0 picks the rotation t;
  * words 1 and 2 pick two spot indices among that rotation's spots (both
    detectors);
  * a pair with a == b yields nothing.
Candidates are ordered by (pair k, m_a, m_b).

Features of a candidate (inputs of the learned proposal; 14 from the pair
itself, 2 cheap-support counts added elsewhere):
   0 cos angle(n_a, n_b)         1 cos angle(w_a, w_b)
   2 |angle difference| / delta  3 sin theta_a
   4 sin theta_b                 5 (lambda_a - lmin)/(lmax - lmin)
   6 same for b                  7 N_a / N_max
   8 N_b / N_max                 9 |p_a - p_b| (lab) / (2 l)
  10 |(p1, p2)_a| / l            11 same for b
  12 detector of a               13 detector of b
"""
from __future__ import annotations

import numpy as np

from . import crystal, mstep, philox
from .crystal import R_to_quat

STREAM_PAIR = 5
E = np.array([1.0, 0.0, 0.0])


def family_representatives(planes):
    """One plane per orbit of the 24 proper cubic rotations, the first in list order."""
    hkl = planes["hkl"]
    index = {tuple(v): i for i, v in enumerate(hkl.tolist())}
    covered = np.zeros(len(hkl), dtype=bool)
    reps = []
    G = np.rint(crystal.cubic_group()).astype(np.int64)
    for m in range(len(hkl)):
        if covered[m]:
            continue
        reps.append(m)
        for S in G:
            covered[index[tuple((S @ hkl[m]).tolist())]] = True
    return np.array(reps, dtype=np.int64)


def spot_normals(geom, p12, block):
    """Sample-frame plane normal n and sin(theta) of detected spots, grain at x = 0."""
    block = np.asarray(block)
    det = block % geom.n_det
    t = block // geom.n_det
    p = geom.det_center[det] + p12[:, :1] * geom.det_a1[det] + p12[:, 1:2] * geom.det_a2[det]
    rh = p / np.linalg.norm(p, axis=1, keepdims=True)
    d = E - rh
    nd = np.linalg.norm(d, axis=1)
    u = d / np.where(nd > 0, nd, 1.0)[:, None]
    n = np.einsum("jba,jb->ja", geom.G[t], u)            # Gamma_t^T u
    return n, nd / 2.0, p


def draw_pairs(geom, obs_off, n_pairs, seed):
    """Pair k -> (a, b) global detected-spot indices, or -1 when a == b / empty rotation."""
    k = np.arange(n_pairs)
    x0, x1, x2, _ = philox.philox4x32_10(k, 0, 0, STREAM_PAIR, *philox.seed_key(seed))
    t = (x0 % np.uint64(geom.n_rot)).astype(np.int64)
    lo = obs_off[t * geom.n_det]
    hi = obs_off[(t + 1) * geom.n_det]
    cnt = (hi - lo).astype(np.uint64)
    safe = np.maximum(cnt, np.uint64(1))
    a = lo + (x1 % safe).astype(np.int64)
    b = lo + (x2 % safe).astype(np.int64)
    bad = (cnt == 0) | (a == b)
    return np.where(bad, -1, a), np.where(bad, -1, b), t


def generate(planes, geom, p12, obs_off, n_pairs, seed, delta_deg=1.5, l_side=200.0, pairs=None):
    """All hypotheses of the first n_pairs pairs (or of the explicit pairs
    (a, b); a pair whose spots are out of range or of two rotations yields
    nothing).  Returns dict of arrays."""
    block = np.repeat(np.arange(geom.n_blocks), np.diff(obs_off))
    n, sth, plab = spot_normals(geom, p12, block)
    w, d, nsq = planes["w"], planes["d"], planes["nsq"]
    reps = family_representatives(planes)
    if pairs is None:
        a_idx, b_idx, _ = draw_pairs(geom, obs_off, n_pairs, seed)
    else:
        a_idx, b_idx = (np.asarray(v, dtype=np.int64).copy() for v in pairs)
        n_pairs = len(a_idx)
        n_obs = len(block)
        valid = (a_idx >= 0) & (b_idx >= 0) & (a_idx < n_obs) & (b_idx < n_obs)
        ta = np.where(valid, block[np.clip(a_idx, 0, max(n_obs - 1, 0))] // geom.n_det, -1)
        tb = np.where(valid, block[np.clip(b_idx, 0, max(n_obs - 1, 0))] // geom.n_det, -2)
        a_idx[ta != tb] = -1
    delta = np.radians(delta_deg)
    ang_w = np.arccos(np.clip(w @ w.T, -1.0, 1.0))
    out = {k: [] for k in ("pair", "ma", "mb", "q", "feat", "a", "b")}
    lmin, lmax = geom.lam_min, geom.lam_max
    nmax = nsq.max()
    for k in range(n_pairs):
        a, b = a_idx[k], b_idx[k]
        if a < 0:
            continue
        la = 2.0 * d * sth[a]
        lb = 2.0 * d * sth[b]
        ina = (la >= lmin) & (la <= lmax)
        inb = (lb >= lmin) & (lb <= lmax)
        cab = float(np.clip(n[a] @ n[b], -1.0, 1.0))
        ang_n = np.arccos(cab)
        for ma in reps:
            if not ina[ma]:
                continue
            ok = inb & (np.abs(ang_w[ma] - ang_n) <= delta)
            par = np.abs(np.abs(w @ w[ma]) - 1.0) < 1e-9
            for mb in np.nonzero(ok & ~par)[0]:
                ca = np.cross(n[a], n[b])
                cw = np.cross(w[ma], w[mb])
                A = np.stack([n[a], n[b], ca / np.linalg.norm(ca)])
                B = np.stack([w[ma], w[mb], cw / np.linalg.norm(cw)])
                R = mstep.wahba(A, B, np.ones(3))
                out["pair"].append(k)
                out["ma"].append(ma)
                out["mb"].append(mb)
                out["a"].append(a)
                out["b"].append(b)
                out["q"].append(R_to_quat(R))
                da, db = block[a] % geom.n_det, block[b] % geom.n_det
                out["feat"].append([
                    cab, float(w[ma] @ w[mb]), abs(ang_w[ma, mb] - ang_n) / delta, sth[a], sth[b],
                    (la[ma] - lmin) / (lmax - lmin), (lb[mb] - lmin) / (lmax - lmin),
                    nsq[ma] / nmax, nsq[mb] / nmax,
                    np.linalg.norm(plab[a] - plab[b]) / (2.0 * l_side),
                    np.linalg.norm(p12[a]) / l_side, np.linalg.norm(p12[b]) / l_side,
                    float(da), float(db)])
    res = {k: np.array(v) for k, v in out.items()}
    if len(res["pair"]) == 0:
        res["q"] = np.zeros((0, 4))
        res["feat"] = np.zeros((0, 14))
    return res
