"""Sparse assignment: each detected spot keeps only its rho nearest model spots
(paper Sec. 5.2, working with sparse assignment matrices; Sec. 7 uses
rho = 32).

Test infrastructure: FP64, plain NumPy.

The paper states the approximation as setting a null assignment weight in
the full plan Q outside the neighbour sets.  Reading (the paper does not say
whose neighbours): the neighbours of detected spot i are the rho model spots j
of its own (rotation, detector) block with the smallest costs c_ij (all of
them if the block has fewer), ties to the lower model-spot index.  The sparse
problem is then the dense one with c_ij = +inf outside the sets, so the
Sinkhorn, marginals and assignments of oracle/sinkhorn.py apply unchanged:
exp(-inf) = 0 is exactly the null weight.  The bins (outlier column, unmatched
row) are kept in full.

The paper ties the first temperature to the farthest neighbour ("non-negligible
probability at start").  Reading: eps_init = median_i c_{i,(rho)} / ln(100),
the temperature at which the farthest neighbour of the median detected spot
weighs 1% of a perfect match.
"""
from __future__ import annotations

import math

import numpy as np

from . import sinkhorn


def neighbours(C, rho):
    """Per row of the cost block C [I_b, J_b]: the indices (into the block's
    columns) of its min(rho, J_b) smallest costs, ordered by (cost, index)."""
    C = np.asarray(C, dtype=np.float64)
    k = min(int(rho), C.shape[1])
    if k == 0:
        return np.zeros((C.shape[0], 0), dtype=np.int64)
    order = np.lexsort((np.broadcast_to(np.arange(C.shape[1]), C.shape), C), axis=1)
    return order[:, :k]


def masked_blocks(C_blocks, rho):
    """The cost blocks with +inf outside each row's neighbour set."""
    out = []
    for C in C_blocks:
        C = np.asarray(C, dtype=np.float64)
        M = np.full(C.shape, np.inf)
        nb = neighbours(C, rho)
        rows = np.repeat(np.arange(C.shape[0]), nb.shape[1])
        M[rows, nb.ravel()] = C[rows, nb.ravel()]
        out.append(M)
    return out


def masked_problem(P, rho):
    """The sparse problem of the dense problem P (same bins and masses)."""
    return sinkhorn.Problem(masked_blocks(P.C, rho), P.c_out, P.c_unm, P.c_sink, P.t_b)


def farthest_costs(C_blocks, rho):
    """c_{i,(rho)} of every row (the cost of its farthest kept neighbour; rows
    of blocks without model spots are left out)."""
    out = []
    for C in C_blocks:
        C = np.asarray(C, dtype=np.float64)
        if C.shape[1] == 0 or C.shape[0] == 0:
            continue
        nb = neighbours(C, rho)
        out.append(C[np.arange(C.shape[0]), nb[:, -1]])
    return np.concatenate(out) if out else np.zeros(0)


def eps_init(C_blocks, rho):
    """First temperature: the median farthest-neighbour cost over ln(100)."""
    far = farthest_costs(C_blocks, rho)
    return float(np.median(far) / math.log(100.0)) if len(far) else 1.0
