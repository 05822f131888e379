"""Prototype scoring of the oracle: single-grain refinement, the unmatched
filter, the SPOT grain-to-spot matrix, greedy selection and the number of
prototypes (paper Sec. 6, App. D-E, Algs. SingleLaueOT and LaueSpotGreedy).

Test infrastructure: FP64, plain NumPy.

Single-grain fitting (App. D, Eq. elbo_single): the column constraint is
dropped, so the assignment of a detected spot is a softmax over the
candidate's model spots of its block and the outlier column:
    Q_ij = exp(-c_ij/eps) / (sum_{j' in J_n, blk(i)} exp(-c_ij'/eps) + exp(-c_out/eps))
(Alg. SingleLaueOT's K diag(a / K1) read as diag(a / K1) K, i.e. rows sum to
a_i).  The paper's schedule (App. D) is the multigrain annealing rule with a
fixed count k_max: eps_init cool^k, k < k_max (cooling_schedule), with four
M-step steps per iteration.  Default reading, measured faster for the same
grains: k_refine iterations on a geometric temperature schedule
30 sigma^2 -> 1.11 sigma^2 (the paper fixes no single-grain schedule; a
start at 30 sigma^2 rather than the multi-grain EM's 111 sigma^2 keeps the
wide first kernels from pulling a candidate onto the clutter around it),
each an E-step followed by k_gn Gauss-Newton steps with Q fixed (the M-step
of oracle/mstep.py; default one step, since with Q fixed a second step moves
the candidate by a negligible amount); the model-spot set of a candidate is
frozen at its start.

Unmatched filter (Sec. 6.2, Sec. 7): a model spot is unmatched when no
detected spot of its block lies within the 3-sigma outlier cost (min_i c_ij >
c_out); a candidate is kept when its unmatched fraction is < f_out.

SPOT (App. E): Lbar_in = log sum_{j in J_n} p(s_i, Z_ij = 1), which up to a
constant shared by all candidates is LSE_j(-c_ij / (2 sigma^2)) over the
candidate's model spots of the detected spot's block.  Reading of the shift
||Lbar||_inf + Lbar: the set function with a floor at the outlier level
phi = -c_out / (2 sigma^2),
    f(S) = sum_i max(phi, max_{n in S} Lbar_in) - |I| phi,
which keeps f(empty) = 0, is monotone and submodular, and makes Lbar sparse
(only entries above phi matter).  Greedy (Alg. LaueSpotGreedy) adds the
candidate of largest increment (lowest index on ties) and records the
increments Delta_k; reading of Eq. spot_ngrains: its second difference
f_{k+1} + f_{k-1} - 2 f_k is the change of the increment, <= 0 for the
submodular f; k* is where f bends most, the largest drop of the increment,
measured over H = 8 picks on each side (the increments of a long run of true
grains vary by about 1% from pick to pick, so the step-1 difference can peak
among the first picks; see n_prototypes).
"""
from __future__ import annotations

import math

import numpy as np

from . import cost, em, forward, mstep, sinkhorn


REFINE_HOT = 30.0     # first temperature of the refinement, in sigma^2
REFINE_COLD = 1.11    # last temperature, in sigma^2


def refine_schedule(sigma, k_refine):
    if k_refine == 1:
        return [REFINE_HOT * sigma ** 2]
    return list(np.geomspace(REFINE_HOT * sigma ** 2, REFINE_COLD * sigma ** 2, k_refine))


def cooling_schedule(eps_init, k_max, cool=0.97):
    """Alg. SingleLaueOT's temperatures: a fixed number k_max of iterations,
    the temperature multiplied by cool after each (App. D: the same annealing
    rule as the multigrain fit, Sec. 5.1 and Sec. 7)."""
    if k_max < 1 or not (0.0 < cool <= 1.0) or eps_init <= 0.0:
        raise ValueError("need k_max >= 1, 0 < cool <= 1 and a positive temperature")
    out = [float(eps_init)]
    for _ in range(int(k_max) - 1):
        out.append(out[-1] * cool)
    return out


def _blocks_costs(planes, geom, distance, p12, obs_off, model, q, x):
    C, ev, vloc = em.build_costs(planes, geom, distance, p12, obs_off, model, q, x)
    return C


def _pairs_single(planes, geom, p_lab, obs_off, model, Qb):
    return em.grain_pairs(planes, geom, p_lab, obs_off, model, Qb, 1)[0]


def refine(planes, geom, distance, p12, obs_off, q, x, sigma, c_out, k_refine=8, k_gn=1, eps_list=None):
    """Single-grain fit of one candidate from (q, x).  eps_list replaces the
    default schedule (e.g. cooling_schedule, with k_gn = 4 for the paper's
    four steps per iteration).  Returns (q, x, model)."""
    q = np.array(q, dtype=np.float64)
    x = np.array(x, dtype=np.float64)
    model = forward.enumerate_visible(planes, q[None], x[None], geom)
    model["offsets"] = forward.block_offsets(model["block"], geom.n_blocks)
    if len(model["m"]) == 0:
        return q, x, model
    p_lab = em.obs_lab(geom, p12, np.repeat(np.arange(geom.n_blocks), np.diff(obs_off)))
    for eps in (refine_schedule(sigma, k_refine) if eps_list is None else eps_list):
        C = _blocks_costs(planes, geom, distance, p12, obs_off, model, q[None], x[None])
        Qb = []
        for Cb in C:
            if Cb.shape[1] == 0:
                Qb.append(np.zeros_like(Cb))
                continue
            ex = np.exp(-Cb / eps)
            z = ex.sum(axis=1, keepdims=True) + math.exp(-c_out / eps)
            Qb.append(ex / z)
        pr = _pairs_single(planes, geom, p_lab, obs_off, model, Qb)
        if pr is None:
            break
        for _ in range(k_gn):
            q, x, *_ = mstep.gn_step(pr, q, x, geom, distance)
    return q, x, model


def score(planes, geom, distance, p12, obs_off, model, q, x, sigma, c_out):
    """Unmatched count and the sparse SPOT column of one candidate at (q, x).

    Returns (n_unmatched, n_model, rows [k], lbar [k]) with lbar > phi."""
    if len(model["m"]) == 0:
        return 0, 0, np.zeros(0, np.int64), np.zeros(0)
    C = _blocks_costs(planes, geom, distance, p12, obs_off, model, np.asarray(q)[None], np.asarray(x)[None])
    phi = -c_out / (2.0 * sigma ** 2)
    unmatched = 0
    rows, vals = [], []
    for b, Cb in enumerate(C):
        if Cb.shape[1] == 0:
            continue
        if Cb.shape[0] == 0:
            unmatched += Cb.shape[1]
            continue
        unmatched += int(np.sum(Cb.min(axis=0) > c_out))
        lb = sinkhorn.lse(-Cb / (2.0 * sigma ** 2), axis=1)
        keep = np.nonzero(lb > phi)[0]
        rows.append(obs_off[b] + keep)
        vals.append(lb[keep])
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    vals = np.concatenate(vals) if vals else np.zeros(0)
    return unmatched, len(model["m"]), rows, vals


def spot_value(cols, n_rows, phi, subset):
    """f(S) = sum_i max(phi, max_{n in S} Lbar_in) - |I| phi for a sparse Lbar.

    cols: list over candidates of (rows, lbar)."""
    cur = np.full(n_rows, phi)
    for n in subset:
        r, v = cols[n]
        np.maximum.at(cur, r, v)
    return float(np.sum(cur - phi))


def greedy(cols, n_rows, phi, k_max=None):
    """Plain greedy (Alg. LaueSpotGreedy): picks and increments Delta_k."""
    cur = np.full(n_rows, phi)
    avail = list(range(len(cols)))
    picks, gains = [], []
    k_max = len(cols) if k_max is None else min(k_max, len(cols))
    for _ in range(k_max):
        best, arg = 0.0, -1
        for n in avail:
            r, v = cols[n]
            gn = float(np.sum(np.maximum(0.0, v - cur[r]))) if len(r) else 0.0
            if gn > best:
                best, arg = gn, n
        if arg < 0:
            break
        picks.append(arg)
        gains.append(best)
        r, v = cols[arg]
        np.maximum.at(cur, r, v)
        avail.remove(arg)
    return picks, np.array(gains)


PROTOTYPE_STEP = 8


def n_prototypes(gains, h=PROTOTYPE_STEP):
    """k* = argmax_{k>=1} [(f_k - f_{k-m}) / m - (f_{k+h} - f_k) / h], m = min(k, h):
    Eq. spot_ngrains' second difference taken over h picks, i.e. the mean
    increment of the h picks up to k minus that of the h picks after it
    (increments beyond the K picks are 0, f_j = f_K for j > K); the lowest k on
    ties.  h = 1 is the printed step (the largest drop Delta_k - Delta_{k+1}).
    f is the running sum of the increments in pick order (FP64)."""
    K = len(gains)
    if K == 0:
        return 0
    f = np.zeros(K + 1)
    for k in range(K):
        f[k + 1] = f[k] + float(gains[k])
    best, arg = -math.inf, 1
    for k in range(1, K + 1):
        m = min(k, h)
        v = (f[k] - f[k - m]) / m - (f[min(K, k + h)] - f[k]) / h
        if v > best:
            best, arg = v, k
    return arg
