"""Forward model of the oracle (paper Sec. 3.2-3.3).

Test infrastructure: FP64, plain NumPy.

For plane m (unit normal w_m, spacing d_m), grain n (R_n, x_n) and sample
rotation Gamma_t (Sec. 3.3):
  u      = Gamma_t R_n w_m                               (plane normal in the lab)
  lambda = 2 d_m u.e                                     (Eq. wavelength_lambda)
  r      = (I - 2 u u^T) e                               (Eq. ray_mnt)
  s      = Gamma_t x_n + tau r,  tau = nu.(gamma - Gamma_t x_n) / nu.r   (Eq. s_mnt)
with beam e = (1,0,0).  A spot is kept (Eq. model_spot_cut) when lambda is in
[lambda_min, lambda_max] and ||s - gamma||_inf < l/2.

Readings where the paper is silent or ambiguous:
  * lambda keeps its sign (no abs); of each +-hkl pair at most one is in band.
  * the ray has one direction r = (I - 2uu^T)e and hits detector d only when
    tau > 0 (the +- of Eq. ray_r names which detector is reached).
  * the detector test is evaluated in detector-local coordinates (two in-plane
    unit axes), strictly: max(|s_1|, |s_2|) < l/2.
  * harmonics: [nh,nk,nl] gives exactly the spot of [h,k,l].  The literal
    per-plane set is V; the model-spot set S keeps, per (grain, rotation,
    detector, direction), only the visible plane of lowest order.
Items within 1e-6 A of a band edge or 1e-4 mm of a detector edge are flagged.
"""
from __future__ import annotations

import numpy as np

from . import crystal

E = np.array([1.0, 0.0, 0.0])
LAM_EDGE = 1e-6
DET_EDGE = 1e-4


class Geometry:
    """Scan rotations, detectors and band, all FP64."""

    def __init__(self, n_rot, domega_rad, detectors, lam_min, lam_max, omega0=0.0):
        self.n_rot = int(n_rot)
        self.domega = float(domega_rad)
        self.omega0 = float(omega0)
        self.G = crystal.scan_rotations(self.n_rot, self.domega, self.omega0)
        self.det_center = np.array([dd.center for dd in detectors], dtype=np.float64)
        self.det_normal = np.array([dd.normal for dd in detectors], dtype=np.float64)
        self.det_a1 = np.array([dd.axis1 for dd in detectors], dtype=np.float64)
        self.det_a2 = np.array([dd.axis2 for dd in detectors], dtype=np.float64)
        self.det_half = np.array([dd.size / 2.0 for dd in detectors], dtype=np.float64)
        self.n_det = len(detectors)
        self.lam_min = float(lam_min)
        self.lam_max = float(lam_max)

    @property
    def n_blocks(self):
        return self.n_rot * self.n_det

    @classmethod
    def from_preset(cls, p):
        return cls(p.n_rot, np.deg2rad(p.domega_deg), p.detectors, p.lam_min, p.lam_max)

    def to_local(self, det, P):
        """Detector-local in-plane coordinates of lab points P [...,3] on detector det."""
        rel = P - self.det_center[det]
        return np.stack([np.einsum("...k,...k->...", rel, self.det_a1[det]),
                         np.einsum("...k,...k->...", rel, self.det_a2[det])], axis=-1)

    def to_lab(self, det, p12):
        """Lab point of detector-local coordinates p12 [...,2] on detector det."""
        return (self.det_center[det] + p12[..., :1] * self.det_a1[det]
                + p12[..., 1:2] * self.det_a2[det])


def _rays(planes, q, x, geom):
    """u, lambda, r, y for all (n, t, m): shapes [N,T,M,3], [N,T,M], [N,T,M,3], [N,T,3]."""
    R = crystal.quat_to_R(q)                                   # [N,3,3]
    GR = np.einsum("tab,nbc->ntac", geom.G, R)                 # Gamma_t R_n
    u = np.einsum("ntac,mc->ntma", GR, planes["w"])            # [N,T,M,3]
    ue = u[..., 0]
    lam = 2.0 * planes["d"][None, None, :] * ue
    r = E - 2.0 * ue[..., None] * u
    y = np.einsum("tab,nb->nta", geom.G, x)                    # Gamma_t x_n
    return u, lam, r, y


def enumerate_visible(planes, q, x, geom, merge_harmonics=True):
    """Visible reflections (Eq. model_spot_cut) ordered by (t, d, n, m).

    Returns a dict of arrays with one entry per spot: m, n, t, det, block
    (t*n_det + det), lam, r [.,3], s [.,3], s12 [.,2] (local), tau, flag
    (near an edge), plus 'merged' (bool: kept in the harmonic-merged set S).
    With merge_harmonics the returned set is S, otherwise the literal V."""
    q = np.atleast_2d(q)
    x = np.atleast_2d(x)
    u, lam, r, y = _rays(planes, q, x, geom)
    N, T, M = lam.shape
    inband = (lam >= geom.lam_min) & (lam <= geom.lam_max)
    recs = []
    for d in range(geom.n_det):
        nu, gam = geom.det_normal[d], geom.det_center[d]
        den = r @ nu                                            # [N,T,M]
        num = ((gam[None, None, :] - y) @ nu)[..., None]        # [N,T,1]
        with np.errstate(divide="ignore", invalid="ignore"):
            tau = num / den
        s = y[:, :, None, :] + tau[..., None] * r
        s12 = geom.to_local(d, s)
        inf = np.max(np.abs(s12), axis=-1)
        vis = inband & (tau > 0) & (inf < geom.det_half[d])
        lam_m = np.minimum(np.abs(lam - geom.lam_min), np.abs(lam - geom.lam_max))
        flag = vis & ((lam_m <= LAM_EDGE) | (np.abs(inf - geom.det_half[d]) <= DET_EDGE))
        # flag also items just outside the band or detector that could enter in FP32
        near_out = inband & (tau > 0) & ~vis & (np.abs(inf - geom.det_half[d]) <= DET_EDGE)
        near_band = ~inband & (tau > 0) & (inf < geom.det_half[d]) & (lam_m <= LAM_EDGE)
        recs.append((d, vis, tau, s, s12, flag, near_out | near_band))
    vis_all = np.stack([rc[1] for rc in recs], axis=-1)         # [N,T,M,D]
    prev = planes["harmonic_prev"]
    merged = vis_all.copy()
    for m in range(M):
        a = prev[m]
        while a >= 0:
            merged[:, :, m, :] &= ~vis_all[:, :, a, :]
            a = prev[a]
    out = {k: [] for k in ("m", "n", "t", "det", "lam", "r", "s", "s12", "tau", "flag", "merged")}
    near_edge = []
    for t in range(T):
        for d, vis, tau, s, s12, flag, near in recs:
            keep = merged[:, t, :, d] if merge_harmonics else vis[:, t, :]
            nn, mm = np.nonzero(keep)                           # row-major: n then m
            out["m"].append(mm)
            out["n"].append(nn)
            out["t"].append(np.full(len(mm), t))
            out["det"].append(np.full(len(mm), d))
            out["lam"].append(lam[nn, t, mm])
            out["r"].append(r[nn, t, mm])
            out["s"].append(s[nn, t, mm])
            out["s12"].append(s12[nn, t, mm])
            out["tau"].append(tau[nn, t, mm])
            out["flag"].append(flag[nn, t, mm])
            out["merged"].append(merged[nn, t, mm, d])
            ne_n, ne_m = np.nonzero(near[:, t, :])
            near_edge.extend((int(a), t, int(b), d) for a, b in zip(ne_n, ne_m))
    res = {k: (np.concatenate(v) if len(v) else np.zeros(0)) for k, v in out.items()}
    for k in ("m", "n", "t", "det"):
        res[k] = res[k].astype(np.int64)
    res["flag"] = res["flag"].astype(bool)
    res["merged"] = res["merged"].astype(bool)
    res["block"] = res["t"] * geom.n_det + res["det"]
    res["near_edge"] = near_edge          # (n, t, m, d) just outside, flagged
    return res


def block_offsets(block, n_blocks):
    """CSR offsets of a block-sorted id array."""
    counts = np.bincount(block, minlength=n_blocks)
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def eval_fixed(planes, q, x, geom, m, n, t, det):
    """Forward model on a frozen list of (m, n, t, det) (no filtering).

    Returns r [J,3], y = Gamma_t x_n [J,3], tau [J], s [J,3], s12 [J,2] and the
    ray vector v = s - y = tau r [J,3]."""
    R = crystal.quat_to_R(np.atleast_2d(q))
    x = np.atleast_2d(x)
    G = geom.G[t]                                              # [J,3,3]
    u = np.einsum("jab,jbc,jc->ja", G, R[n], planes["w"][m])
    r = E - 2.0 * u[:, :1] * u
    y = np.einsum("jab,jb->ja", G, x[n])
    nu = geom.det_normal[det]
    gam = geom.det_center[det]
    tau = np.einsum("jk,jk->j", gam - y, nu) / np.einsum("jk,jk->j", r, nu)
    s = y + tau[:, None] * r
    rel = s - gam
    s12 = np.stack([np.einsum("jk,jk->j", rel, geom.det_a1[det]),
                    np.einsum("jk,jk->j", rel, geom.det_a2[det])], axis=1)
    return {"r": r, "y": y, "tau": tau, "s": s, "s12": s12, "v": s - y, "u": u}
