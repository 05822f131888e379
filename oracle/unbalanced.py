"""Unbalanced entropic OT E-step (paper App. C, Problem B; Alg. UnbalancedOT),
one of the two outlier treatments the paper compares its model with.

Test infrastructure: FP64, plain NumPy.

Problem B relaxes both marginals into generalised KL penalties,
  max_Q <L, Q> + eps H(Q) - kappa D(Q 1, a) - lambda D(Q^T 1, b),
with no outlier row or column.  With L = -c (mm^2, so eps, kappa and lambda
are in mm^2 too: a value k in the paper's log-likelihood units is
k * 2 sigma_mm^2 here), a = b = 1 and potentials f = eps log x,
g = eps log y, the algorithm's updates
  x <- (a / K y)^tau_r,   y <- (b / K^T x)^tau_c
read, in the log domain,
  f_i = tau_r * (-eps LSE_j (g_j - c_ij) / eps)        (rows, all at once)
  g_j = tau_c * (-eps LSE_i (f_i - c_ij) / eps)        (columns, with the new f)
Readings:
  * exponents: the text puts kappa on the row (detected-spot) marginal and
    lambda on the column marginal, the printed algorithm the other way round;
    the text is followed: tau_r = kappa / (kappa + eps), tau_c = lambda /
    (lambda + eps);
  * stopping: the algorithm's max(||x' - x||, ||y' - y||) names neither norm
    nor scale; read as the largest change an update makes to a row (column)
    marginal of the plan, S |exp(du / eps) - 1| with S that row's (column's)
    plan mass before the update and du its potential change, after a column
    half, <= tol, or n_max iterations.  It is the balanced rule's |row - 1|
    (the row-marginal error) carried over: an update scales its row by
    exp(du / eps).  A relative change of the scaling alone, |du| / eps, would
    also count spots far from every model spot, whose potentials are large,
    carry no mass and cannot settle below their rounding in FP32;
  * a row (column) with no finite cost (a block without model (detected)
    spots, or no kept entry under a sparse mask) carries no plan mass; its
    potential is set to 0;
  * hard assignment: the plan leaves 1 - sum_j Q_ij of a detected spot's unit
    mass untransported; the spot is an outlier when that deficit exceeds its
    largest entry, else it is assigned to the argmax (lowest index on ties).
At the fixed point the first-order conditions give row_i = a_i exp(-f_i/kappa)
and col_j = b_j exp(-g_j/lambda); kappa, lambda -> inf recovers balanced OT.
"""
from __future__ import annotations

import math

import numpy as np


def _lse_masked(x, finite, axis):
    """log sum exp over the finite entries; -inf where there are none."""
    x = np.where(finite, x, -np.inf)
    m = np.max(x, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        out = np.log(np.sum(np.where(finite, np.exp(x - m), 0.0), axis=axis, keepdims=True)) + m
    return np.squeeze(out, axis=axis)


def _offsets(C_blocks):
    row_off = np.concatenate([[0], np.cumsum([C.shape[0] for C in C_blocks])]).astype(np.int64)
    col_off = np.concatenate([[0], np.cumsum([C.shape[1] for C in C_blocks])]).astype(np.int64)
    return row_off, col_off


def row_update(C_blocks, row_off, col_off, g, eps, tau):
    f = np.zeros(row_off[-1])
    for b, C in enumerate(C_blocks):
        r0, r1 = row_off[b], row_off[b + 1]
        if C.shape[0] == 0 or C.shape[1] == 0:
            continue
        fin = np.isfinite(C)
        gb = g[col_off[b]:col_off[b + 1]]
        s = _lse_masked((gb[None, :] - np.where(fin, C, 0.0)) / eps, fin, axis=1)
        f[r0:r1] = np.where(fin.any(axis=1), -tau * eps * s, 0.0)
    return f


def col_update(C_blocks, row_off, col_off, f, eps, tau):
    g = np.zeros(col_off[-1])
    for b, C in enumerate(C_blocks):
        c0, c1 = col_off[b], col_off[b + 1]
        if C.shape[0] == 0 or C.shape[1] == 0:
            continue
        fin = np.isfinite(C)
        fb = f[row_off[b]:row_off[b + 1]]
        s = _lse_masked((fb[:, None] - np.where(fin, C, 0.0)) / eps, fin, axis=0)
        g[c0:c1] = np.where(fin.any(axis=0), -tau * eps * s, 0.0)
    return g


def mass_change(S, du, eps):
    """max |S exp(du / eps) - S| over rows (columns) with plan mass S before
    an update that changes their potential by du (0 for no rows)."""
    if len(S) == 0:
        return 0.0
    with np.errstate(divide="ignore"):
        logS = np.log(S)
    return float(np.max(np.abs(np.exp(logS + du / eps) - S)))


def solve(C_blocks, eps, kappa, lam, tol=1e-5, n_max=2000, f=None, g=None):
    """Iterations from (f, g) (zeros = the algorithm's x = y = 1).  Returns
    dict with f, g, n_iter, err, row_off, col_off."""
    C_blocks = [np.asarray(C, dtype=np.float64) for C in C_blocks]
    row_off, col_off = _offsets(C_blocks)
    tau_r = kappa / (kappa + eps)
    tau_c = lam / (lam + eps)
    f = np.zeros(row_off[-1]) if f is None else np.array(f, dtype=np.float64)
    g = np.zeros(col_off[-1]) if g is None else np.array(g, dtype=np.float64)
    err = math.inf
    k = 0
    for k in range(1, n_max + 1):
        s_row = marginals(C_blocks, f, g, eps)[0]
        fn = row_update(C_blocks, row_off, col_off, g, eps, tau_r)
        s_col = marginals(C_blocks, fn, g, eps)[1]
        gn = col_update(C_blocks, row_off, col_off, fn, eps, tau_c)
        err = max(mass_change(s_row, fn - f, eps), mass_change(s_col, gn - g, eps))
        f, g = fn, gn
        if err <= tol:
            break
    return {"f": f, "g": g, "n_iter": k, "err": err, "row_off": row_off, "col_off": col_off}


def plan_blocks(C_blocks, f, g, eps):
    """Dense Q blocks (0 where the cost is +inf)."""
    row_off, col_off = _offsets(C_blocks)
    out = []
    for b, C in enumerate(C_blocks):
        C = np.asarray(C, dtype=np.float64)
        fin = np.isfinite(C)
        e = f[row_off[b]:row_off[b + 1], None] + g[None, col_off[b]:col_off[b + 1]] - np.where(fin, C, 0.0)
        out.append(np.exp(np.where(fin, e / eps, -np.inf)))
    return out


def marginals(C_blocks, f, g, eps):
    Q = plan_blocks(C_blocks, f, g, eps)
    rows = np.concatenate([q.sum(axis=1) for q in Q]) if Q else np.zeros(0)
    cols = np.concatenate([q.sum(axis=0) for q in Q]) if Q else np.zeros(0)
    return rows, cols


def hard_assignment(C_blocks, f, g, eps):
    """Per detected spot: (j_star (global model index, -1 = outlier), Q_ij*
    or the deficit, the deficit max(0, 1 - sum_j Q_ij))."""
    row_off, col_off = _offsets(C_blocks)
    n = int(row_off[-1])
    js = np.full(n, -1, dtype=np.int64)
    qs = np.zeros(n)
    qo = np.ones(n)
    for b, q in enumerate(plan_blocks(C_blocks, f, g, eps)):
        r0, r1 = row_off[b], row_off[b + 1]
        if q.shape[0] == 0:
            continue
        qo[r0:r1] = np.maximum(0.0, 1.0 - q.sum(axis=1))
        if q.shape[1] == 0:
            qs[r0:r1] = qo[r0:r1]
            continue
        a = np.argmax(q, axis=1)
        qm = q[np.arange(q.shape[0]), a]
        out = (qo[r0:r1] > qm) | (qm <= 0.0)
        js[r0:r1] = np.where(out, -1, a + col_off[b])
        qs[r0:r1] = np.where(out, qo[r0:r1], qm)
    return js, qs, qo


def primal(C_blocks, Q_blocks, eps, kappa, lam):
    """Problem B's objective as a cost to minimise, for any non-negative plan
    (zero wherever the cost is +inf): <c, Q> - eps H(Q) + kappa KL(Q1 | 1) +
    lambda KL(Q^T 1 | 1), with H(Q) = -sum Q (log Q - 1) and
    KL(p | 1) = sum p log p - p + 1."""
    def xlogx(p):
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(p > 0, p * np.log(np.where(p > 0, p, 1.0)), 0.0)
    lin = ent = 0.0
    rows, cols = [], []
    for C, Q in zip(C_blocks, Q_blocks):
        C = np.asarray(C, dtype=np.float64)
        Q = np.asarray(Q, dtype=np.float64)
        lin += float(np.sum(np.where(Q > 0, Q * np.where(np.isfinite(C), C, 0.0), 0.0)))
        ent += float(np.sum(xlogx(Q) - Q))
        rows.append(Q.sum(axis=1))
        cols.append(Q.sum(axis=0))
    r = np.concatenate(rows) if rows else np.zeros(0)
    c = np.concatenate(cols) if cols else np.zeros(0)
    return lin + eps * ent + kappa * float(np.sum(xlogx(r) - r + 1.0)) + lam * float(np.sum(xlogx(c) - c + 1.0))
