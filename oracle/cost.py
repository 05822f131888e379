"""Pairwise assignment cost of the oracle (paper Sec. 4, Eqs. likelihood / update_L).

Test infrastructure: FP64, plain NumPy.

The paper's likelihood of matching detected spot i to model spot j is
L_ij = sigma^-2 rhat_ij^T r_j with rhat_ij the unit vector from the grain
centre Gamma_t x_n to the detected spot (Sec. 4).  With unit vectors,
rhat^T r = 1 - ||rhat - r||^2 / 2, so up to a constant shared by all pairs
L_ij = -||rhat_ij - r_j||^2 / (2 sigma^2).  Reading: sigma is angular and
equals sigma_mm / D for detector distance D, which turns the likelihood into a
cost in mm^2,
    c_ij = D^2 ||rhat_ij - r_j||^2,     L_ij = const - c_ij / (2 sigma_mm^2),
and an entropic temperature eps_paper on L becomes eps = 2 sigma_mm^2 eps_paper
on c.  Outlier bins (Eq. update_L): the outlier likelihood is the value at an
angular miss of 3 sigma, c_out = 2 D^2 (1 - cos(3 sigma_mm / D)); an unmatched
model spot costs the vMF value at zero angle, c_unm = 0; the sink Q_00 costs
c_out like the outlier column.

Everything is evaluated in a detector-local frame (normal, axis1, axis2):
the detected spot is p = (0, p1, p2), the model spot s = (0, s1, s2) and the
model ray vector v = s - y = tau r (so y = s - v and r = v / |v|).
"""
from __future__ import annotations

import numpy as np


def c_out(sigma_mm, distance, k_sigma=3.0):
    return 2.0 * distance ** 2 * (1.0 - np.cos(k_sigma * sigma_mm / distance))


def chord_cost(p12, s12, v_loc, distance):
    """c_ij = D^2 ||rhat_ij - r_j||^2 for all rows of p12 [I,2] and columns (s12 [J,2], v_loc [J,3])."""
    p = np.zeros((p12.shape[0], 3))
    p[:, 1:] = p12
    s = np.zeros((s12.shape[0], 3))
    s[:, 1:] = s12
    y = s - v_loc                                   # grain centre in the local frame
    dvec = p[:, None, :] - y[None, :, :]            # [I,J,3]
    rhat = dvec / np.linalg.norm(dvec, axis=-1, keepdims=True)
    r = v_loc / np.linalg.norm(v_loc, axis=-1, keepdims=True)
    diff = rhat - r[None, :, :]
    return distance ** 2 * np.einsum("ijk,ijk->ij", diff, diff)


def chord_cost_cosine(p12, s12, v_loc, distance):
    """The same cost through 2 D^2 (1 - rhat.r) (cancels badly; used only as a pin)."""
    p = np.zeros((p12.shape[0], 3))
    p[:, 1:] = p12
    s = np.zeros((s12.shape[0], 3))
    s[:, 1:] = s12
    y = s - v_loc
    dvec = p[:, None, :] - y[None, :, :]
    rhat = dvec / np.linalg.norm(dvec, axis=-1, keepdims=True)
    r = v_loc / np.linalg.norm(v_loc, axis=-1, keepdims=True)
    return 2.0 * distance ** 2 * (1.0 - np.einsum("ijk,jk->ij", rhat, r))


def v_local(geom, det, v_lab):
    """Components of lab vectors v [J,3] along (normal, axis1, axis2) of detector det [J]."""
    return np.stack([np.einsum("jk,jk->j", v_lab, geom.det_normal[det]),
                     np.einsum("jk,jk->j", v_lab, geom.det_a1[det]),
                     np.einsum("jk,jk->j", v_lab, geom.det_a2[det])], axis=1)
