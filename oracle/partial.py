"""Partial entropic OT E-step (paper App. C, Problem A; Alg. PartialOT), the
other outlier treatment the paper compares its model with.

Test infrastructure: FP64, plain NumPy.

Problem A:  max_Q <L, Q> + eps H(Q)  over plans Q >= 0 of the block set,
with Q 1 <= a, Q^T 1 <= b and 1^T Q 1 = m, no outlier row or column.  With
L = -c and a = b = 1 it is the KL projection of the Gibbs kernel
K = exp(-c / eps) onto the intersection of three convex sets, computed by
iterated Bregman projections with Dykstra's corrections for the two
inequality sets (the listing's Q_1, Q_2) and none for the affine mass set
(a correction there is a no-op).  `dykstra` below takes those steps on dense
matrices; `solve` is the same iteration on potentials:
  Q = exp((f_i + g_j + h - c_ij) / eps)
  rows:    f_i = min(0, -eps LSE_j (g_j + h - c_ij) / eps)
  columns: g_j = min(0, -eps LSE_i (f_i + h - c_ij) / eps)
  mass:    h <- h + eps ln(m / M),  M = sum_j min(1, column sum before the column step)
The reduction: started from K with unit corrections, a row step multiplies
row i of K (x) Q_1 by s_i = min(1, 1 / row sum) and sets Q_1's row to 1 / s_i,
so the correction always undoes the accumulated row scaling, i.e.
Q_1 = exp(-f / eps); the row sums of K (x) Q_1 are therefore those of
exp((g + h - c) / eps), independent of f.  The same holds for columns.
Readings:
  * the listing computes row sums of K^k and scales K^k (x) Q_1; Dykstra's
    step projects K^k (x) Q_1 and is read so (the two coincide only at the
    first iteration);
  * the listing's Q_3 and its division by K^k are dropped: the mass set is
    affine, where a Bregman projection needs no correction;
  * mass: the experiments give m_OT as a fraction of the transported mass;
    the mass is m = m_OT * sum_b min(|I_b|, |J_b|), the largest mass plans of
    the block set can carry;
  * start: every solve starts from the Gibbs kernel (f = g = h = 0), as the
    algorithm does; a warm start would project a different matrix;
  * stopping: the listing's ||K - K^prev||_F is read, like the other two
    variants, on marginals: the largest change between consecutive iterates
    of a row mass of the plan entering the row step, or of a column mass of
    the plan entering the column step (with its new row potentials),
    <= tol, checked from the second iteration on;
  * rows (columns) without entries get potential 0; masked (+inf) costs carry
    no mass.
"""
from __future__ import annotations

import math

import numpy as np

from .unbalanced import _lse_masked, _offsets, marginals, plan_blocks


def max_mass(C_blocks):
    """sum_b min(|I_b|, |J_b|)."""
    return float(sum(min(C.shape[0], C.shape[1]) for C in C_blocks))


def _row_lse(C_blocks, row_off, col_off, g, h, eps):
    """LSE_j (g_j + h - c_ij) / eps per row (-inf without entries)."""
    out = np.full(row_off[-1], -np.inf)
    for b, C in enumerate(C_blocks):
        if C.shape[0] == 0 or C.shape[1] == 0:
            continue
        fin = np.isfinite(C)
        gb = g[col_off[b]:col_off[b + 1]]
        out[row_off[b]:row_off[b + 1]] = _lse_masked((gb[None, :] + h - np.where(fin, C, 0.0)) / eps, fin, axis=1)
    return out


def _col_lse(C_blocks, row_off, col_off, f, h, eps):
    out = np.full(col_off[-1], -np.inf)
    for b, C in enumerate(C_blocks):
        if C.shape[0] == 0 or C.shape[1] == 0:
            continue
        fin = np.isfinite(C)
        fb = f[row_off[b]:row_off[b + 1]]
        out[col_off[b]:col_off[b + 1]] = _lse_masked((fb[:, None] + h - np.where(fin, C, 0.0)) / eps, fin, axis=0)
    return out


def solve(C_blocks, eps, m_frac, tol=1e-5, n_max=2000, history=False):
    """Returns dict with f, g (h folded into f, so Q = exp((f + g - c)/eps)),
    h, mass, n_iter, err."""
    C_blocks = [np.asarray(C, dtype=np.float64) for C in C_blocks]
    row_off, col_off = _offsets(C_blocks)
    m = m_frac * max_mass(C_blocks)
    f = np.zeros(row_off[-1])
    g = np.zeros(col_off[-1])
    h = 0.0
    rho_prev = kap_prev = None
    err = math.inf
    k = 0
    errs = []
    for k in range(1, n_max + 1):
        ls = _row_lse(C_blocks, row_off, col_off, g, h, eps)
        with np.errstate(invalid="ignore"):
            rho = np.where(np.isfinite(ls), np.exp(ls + f / eps), 0.0)        # row masses of the current plan
        f = np.where(np.isfinite(ls), np.minimum(0.0, -eps * ls), 0.0)
        ls = _col_lse(C_blocks, row_off, col_off, f, h, eps)
        with np.errstate(invalid="ignore"):
            kap = np.where(np.isfinite(ls), np.exp(ls + g / eps), 0.0)        # column masses before the column step
            M = float(np.sum(np.where(np.isfinite(ls), np.exp(np.minimum(ls, 0.0)), 0.0)))
        g = np.where(np.isfinite(ls), np.minimum(0.0, -eps * ls), 0.0)
        if M > 0.0:
            h += eps * math.log(m / M)
        if rho_prev is not None:
            err = max(float(np.max(np.abs(rho - rho_prev))) if len(rho) else 0.0,
                      float(np.max(np.abs(kap - kap_prev))) if len(kap) else 0.0)
        rho_prev, kap_prev = rho, kap
        errs.append(err)
        if err <= tol:
            break
    out = {"f": f + h, "g": g, "h": h, "mass": m, "n_iter": k, "err": err,
           "row_off": row_off, "col_off": col_off}
    if history:
        out["errs"] = errs
    return out


def dykstra(C, eps, m, n_iter):
    """Dykstra's iterated Bregman projections on one dense finite block C
    (the listing's steps with the readings above): returns the plan."""
    C = np.asarray(C, dtype=np.float64)
    K = np.exp(-C / eps)
    Q1 = np.ones_like(K)
    Q2 = np.ones_like(K)
    for _ in range(n_iter):
        KQ = K * Q1
        K1 = np.minimum(1.0 / KQ.sum(axis=1), 1.0)[:, None] * KQ
        Q1 = KQ / K1
        KQ = K1 * Q2
        K2 = KQ * np.minimum(1.0 / KQ.sum(axis=0), 1.0)[None, :]
        Q2 = KQ / K2
        K = K2 * (m / K2.sum())
    return K


def hard_assignment(C_blocks, f, g, eps):
    """As for unbalanced OT: the untransported mass 1 - sum_j Q_ij plays the
    outlier column's part."""
    from .unbalanced import hard_assignment as ha
    return ha(C_blocks, f, g, eps)


__all__ = ["solve", "dykstra", "max_mass", "plan_blocks", "marginals", "hard_assignment"]
