"""Entropic OT E-step with outlier row and column (paper Sec. 4.2-4.3, Eqs.
update_L, elbo, estep_obj; Alg. BalancedOT), in the log domain.

Test infrastructure: FP64, plain NumPy.

The plan Q is (|I|+1) x (|J|+1): rows are detected spots plus row 0, columns
are model spots plus column 0.  Q_ij may be non-zero only for a detected and a
model spot of the same (rotation, detector) block (Sec. 4.1, set Q; pairs on
different detectors have costs so large that exp(-c/eps) is exactly 0 at the
temperatures used).  Costs (see oracle/cost.py): c_ij inside blocks, c_i0 =
c_out (detected spot i is an outlier), c_0j = c_unm (model spot j unmatched),
c_00 = c_sink.  Marginals: a_i = b_j = 1; readings of Sec. 4.3: row 0 carries
the user-controlled T_b (maximum number of unmatched model spots), column 0
carries T_a = T_b + |I| - |J| so that both sides hold the same mass.

Alg. BalancedOT alternates x <- a / (K y), y <- b / (K^T x) with K = exp(L/eps)
from x = y = 1.  With f = eps log x, g = eps log y and L = -c this is
  f_i = eps log a_i - eps LSE_j (g_j - c_ij)/eps      (row half, all rows at once)
  g_j = eps log b_j - eps LSE_i (f_i - c_ij)/eps      (column half, with the new f)
and Q_ij = exp((f_i + g_j - c_ij)/eps).  The paper leaves the stopping norm
open; reading: stop after the first column half at which the largest relative
row-marginal error is <= tol, or after n_max iterations.
"""
from __future__ import annotations

import math

import numpy as np


def lse(x, axis=None):
    """log(sum(exp(x))) with the maximum shifted out."""
    x = np.asarray(x, dtype=np.float64)
    m = np.max(x, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    out = np.log(np.sum(np.exp(x - m), axis=axis, keepdims=True)) + m
    return np.squeeze(out, axis=axis) if axis is not None else float(out.squeeze())


class Problem:
    """Block-structured OT problem.  C[b] is the [I_b, J_b] cost block b."""

    def __init__(self, C_blocks, c_out, c_unm, c_sink, t_b):
        self.C = [np.asarray(c, dtype=np.float64) for c in C_blocks]
        self.ni = np.array([c.shape[0] for c in self.C])
        self.nj = np.array([c.shape[1] for c in self.C])
        self.row_off = np.concatenate([[0], np.cumsum(self.ni)])
        self.col_off = np.concatenate([[0], np.cumsum(self.nj)])
        self.I = int(self.row_off[-1])
        self.J = int(self.col_off[-1])
        self.c_out, self.c_unm, self.c_sink = float(c_out), float(c_unm), float(c_sink)
        self.t_b = float(t_b)
        self.t_a = self.t_b + self.I - self.J
        if self.t_a < 0:
            raise ValueError("infeasible masses: T_b + |I| - |J| < 0")


def default_tb(n_model, frac=0.4):
    """T_b = ceil(0.4 |J|) (Sec. 7 parameters)."""
    return float(math.ceil(frac * n_model))


def row_half(P, g, g0, eps):
    f = np.empty(P.I)
    for b, C in enumerate(P.C):
        r0, r1 = P.row_off[b], P.row_off[b + 1]
        gb = g[P.col_off[b]:P.col_off[b + 1]]
        ex = np.concatenate([(gb[None, :] - C) / eps,
                             np.full((C.shape[0], 1), (g0 - P.c_out) / eps)], axis=1)
        f[r0:r1] = eps * math.log(1.0) - eps * lse(ex, axis=1)
    f0 = eps * math.log(P.t_b) - eps * lse(np.concatenate([(g - P.c_unm) / eps,
                                                          [(g0 - P.c_sink) / eps]]))
    return f, f0


def col_half(P, f, f0, eps):
    g = np.empty(P.J)
    for b, C in enumerate(P.C):
        c0, c1 = P.col_off[b], P.col_off[b + 1]
        fb = f[P.row_off[b]:P.row_off[b + 1]]
        ex = np.concatenate([(fb[:, None] - C) / eps,
                             np.full((1, C.shape[1]), (f0 - P.c_unm) / eps)], axis=0)
        g[c0:c1] = eps * math.log(1.0) - eps * lse(ex, axis=0)
    g0 = eps * math.log(P.t_a) - eps * lse(np.concatenate([(f - P.c_out) / eps,
                                                          [(f0 - P.c_sink) / eps]]))
    return g, g0


def plan_blocks(P, f, g, eps):
    """Dense Q blocks [I_b, J_b] of the matched part."""
    out = []
    for b, C in enumerate(P.C):
        fb = f[P.row_off[b]:P.row_off[b + 1]]
        gb = g[P.col_off[b]:P.col_off[b + 1]]
        out.append(np.exp((fb[:, None] + gb[None, :] - C) / eps))
    return out


def marginals(P, f, g, f0, g0, eps):
    """Row sums (incl. row 0) and column sums (incl. column 0) of the full plan."""
    Qb = plan_blocks(P, f, g, eps)
    q_i0 = np.exp((f + g0 - P.c_out) / eps)
    q_0j = np.exp((f0 + g - P.c_unm) / eps)
    q_00 = math.exp((f0 + g0 - P.c_sink) / eps)
    rows = np.concatenate([q.sum(axis=1) for q in Qb]) + q_i0
    cols = np.concatenate([q.sum(axis=0) for q in Qb]) + q_0j
    row0 = q_0j.sum() + q_00
    col0 = q_i0.sum() + q_00
    return rows, row0, cols, col0


def row_error(P, f, g, f0, g0, eps):
    rows, row0, _, _ = marginals(P, f, g, f0, g0, eps)
    err = np.max(np.abs(rows - 1.0)) if P.I else 0.0
    return max(float(err), abs(row0 - P.t_b) / P.t_b if P.t_b > 0 else 0.0)


def solve(P, eps, tol=1e-5, n_max=2000, f=None, g=None, f0=0.0, g0=0.0, history=False):
    """Sinkhorn iterations from potentials (f, g, f0, g0) (zeros = Alg. BalancedOT's x=y=1),
    re-centred on entry so that f0 = 0 (the same plan and dual value).

    Returns dict with f, g, f0, g0, n_iter, err (and per-iteration dual values
    if history)."""
    f = np.zeros(P.I) if f is None else np.array(f, dtype=np.float64)
    g = np.zeros(P.J) if g is None else np.array(g, dtype=np.float64)
    f0, g0 = float(f0), float(g0)
    # gauge: the plan depends on the potentials only through f_i + g_j, f_i +
    # g_0, f_0 + g_j and f_0 + g_0, so (f - C, g + C, f_0 - C, g_0 + C) is the
    # same state; a warm start is re-centred with C = f_0 (f_0 = 0 on entry)
    if math.isfinite(f0) and f0 != 0.0:
        f, g, g0, f0 = f - f0, g + f0, g0 + f0, 0.0
    hist = []
    err = math.inf
    k = 0
    for k in range(1, n_max + 1):
        f, f0 = row_half(P, g, g0, eps)
        g, g0 = col_half(P, f, f0, eps)
        err = row_error(P, f, g, f0, g0, eps)
        if history:
            hist.append(dual_value(P, f, g, f0, g0, eps))
        if err <= tol:
            break
    return {"f": f, "g": g, "f0": f0, "g0": g0, "n_iter": k, "err": err, "dual": hist}


def dual_value(P, f, g, f0, g0, eps):
    """Entropic dual sum a.f + b.g - eps * (total plan mass) (maximised by Sinkhorn)."""
    rows, row0, _, _ = marginals(P, f, g, f0, g0, eps)
    mass = rows.sum() + row0
    return float(f.sum() + P.t_b * f0 + g.sum() + P.t_a * g0 - eps * mass)


def objectives(P, f, g, f0, g0, eps, sigma_mm=None, distance=None):
    """FP64 summaries of a plan: inlier cost <c,Q>, total cost incl. bins,
    entropy H(Q) = -sum Q log Q, and (if sigma and D given) the paper-unit sEM
    objective <L,Q> + eps_p H(Q) with L = kappa - c / (2 sigma^2)."""
    Qb = plan_blocks(P, f, g, eps)
    # masked entries (c = +inf, sparse assignment) carry no mass: their terms are 0
    inl = sum(float(np.sum(np.where(q > 0, q * np.where(np.isfinite(c), c, 0.0), 0.0))) for q, c in zip(Qb, P.C))
    q_i0 = np.exp((f + g0 - P.c_out) / eps)
    q_0j = np.exp((f0 + g - P.c_unm) / eps)
    q_00 = math.exp((f0 + g0 - P.c_sink) / eps)
    tot = inl + P.c_out * q_i0.sum() + P.c_unm * q_0j.sum() + P.c_sink * q_00

    def ent(qv, logq):
        return -float(np.sum(np.where(qv > 0, qv * np.where(np.isfinite(logq), logq, 0.0), 0.0)))
    H = sum(ent(q, (f[P.row_off[b]:P.row_off[b + 1], None] + g[None, P.col_off[b]:P.col_off[b + 1]] - P.C[b]) / eps)
            for b, q in enumerate(Qb))
    H += ent(q_i0, (f + g0 - P.c_out) / eps) + ent(q_0j, (f0 + g - P.c_unm) / eps)
    H += ent(np.array([q_00]), np.array([(f0 + g0 - P.c_sink) / eps]))
    out = {"cost_inlier": inl, "cost_total": tot, "entropy": H,
           "mass": float(sum(q.sum() for q in Qb) + q_i0.sum() + q_0j.sum() + q_00)}
    if sigma_mm is not None and distance is not None:
        kappa = (distance / sigma_mm) ** 2
        mass = out["mass"]
        out["sem_objective"] = kappa * mass - tot / (2.0 * sigma_mm ** 2) + eps / (2.0 * sigma_mm ** 2) * H
    return out


def hard_assignment(P, f, g, f0, g0, eps):
    """Per detected spot: argmax over its block's model spots and the outlier
    column (index -1), lowest index on ties; returns (j_star, Q_ij*, Q_i0)."""
    js = np.empty(P.I, dtype=np.int64)
    qs = np.empty(P.I)
    q_i0 = np.exp((f + g0 - P.c_out) / eps)
    for b, q in enumerate(plan_blocks(P, f, g, eps)):
        r0, r1 = P.row_off[b], P.row_off[b + 1]
        if q.shape[1] == 0:
            js[r0:r1] = -1
            qs[r0:r1] = q_i0[r0:r1]
            continue
        a = np.argmax(q, axis=1)
        qm = q[np.arange(q.shape[0]), a]
        out = q_i0[r0:r1] > qm
        js[r0:r1] = np.where(out, -1, a + P.col_off[b])
        qs[r0:r1] = np.where(out, q_i0[r0:r1], qm)
    return js, qs, q_i0
