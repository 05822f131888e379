"""Pins of the oracle cost and Sinkhorn E-step: identities, closed forms,
marginal constraints, monotone dual and brute-force assignment as eps -> 0."""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import cost, sinkhorn

D = 150.0


def _cols(rng, n):
    s12 = rng.uniform(-80, 80, (n, 2))
    y = np.c_[np.full(n, -150.0), rng.uniform(-2, 2, (n, 2))]     # grain centre, local frame
    y[:, 0] += rng.uniform(-2, 2, n)
    v = np.c_[np.zeros(n), s12] - y
    return s12, v


def test_chord_cost_identities():
    rng = np.random.default_rng(0)
    s12, v = _cols(rng, 7)
    p12 = s12[[0, 3, 5]] + rng.normal(0, 0.5, (3, 2))
    c = cost.chord_cost(p12, s12, v, D)
    assert np.all(c >= 0)
    # zero exactly on the model spot
    assert np.allclose(cost.chord_cost(s12, s12, v, D).diagonal(), 0.0, atol=1e-18)
    # equals 2 D^2 (1 - cos) in FP64, away from tiny angles
    c2 = cost.chord_cost_cosine(p12, s12, v, D)
    assert np.allclose(c, c2, rtol=1e-9)
    # independent check: squared angle for small separations, in mm^2 at distance D
    pp = np.c_[np.zeros(3), p12]
    y = np.c_[np.zeros(7), s12] - v
    for i in range(3):
        for j in range(7):
            a = pp[i] - y[j]
            ang = math.atan2(np.linalg.norm(np.cross(a, v[j])), a @ v[j])
            assert c[i, j] == pytest.approx(2 * D * D * (1 - math.cos(ang)), rel=1e-10)


def test_c_out_is_three_sigma():
    # 3 sigma of angular noise sigma_mm/D: c_out ~ 9 sigma^2 for small angles
    assert cost.c_out(1.0, 150.0) == pytest.approx(9.0, rel=1e-4)
    assert cost.c_out(0.3, 150.0) == pytest.approx(0.81, rel=1e-4)


def _problem(rng, sizes, c_out=2.0, t_frac=0.4, spread=3.0):
    C = [rng.uniform(0, spread, s) for s in sizes]
    J = sum(s[1] for s in sizes)
    return sinkhorn.Problem(C, c_out, 0.0, c_out, math.ceil(t_frac * J))


def test_marginals_at_convergence():
    rng = np.random.default_rng(1)
    P = _problem(rng, [(5, 4), (3, 6), (0, 2), (4, 0), (7, 7)])
    sol = sinkhorn.solve(P, 0.5, tol=1e-12, n_max=20000)
    rows, row0, cols, col0 = sinkhorn.marginals(P, sol["f"], sol["g"], sol["f0"], sol["g0"], 0.5)
    assert np.allclose(rows, 1.0, atol=1e-11)
    assert np.allclose(cols, 1.0, atol=1e-11)
    assert row0 == pytest.approx(P.t_b, abs=1e-10)
    assert col0 == pytest.approx(P.t_a, abs=1e-10)
    assert P.t_a == P.t_b + P.I - P.J


def test_constant_cost_gives_product_plan():
    # all costs equal (bins included): the plan is the product a b^T / total mass
    P = sinkhorn.Problem([np.full((6, 8), 2.0)], 2.0, 2.0, 2.0, 4)
    sol = sinkhorn.solve(P, 0.7, tol=1e-13, n_max=5000)
    a = np.r_[np.ones(6), P.t_b]
    b = np.r_[np.ones(8), P.t_a]
    Q = np.zeros((7, 9))
    Q[:6, :8] = sinkhorn.plan_blocks(P, sol["f"], sol["g"], 0.7)[0]
    Q[:6, 8] = np.exp((sol["f"] + sol["g0"] - 2.0) / 0.7)
    Q[6, :8] = np.exp((sol["f0"] + sol["g"] - 2.0) / 0.7)
    Q[6, 8] = math.exp((sol["f0"] + sol["g0"] - 2.0) / 0.7)
    assert np.allclose(Q, np.outer(a, b) / a.sum(), atol=1e-10)


def test_large_eps_approaches_product_plan():
    rng = np.random.default_rng(2)
    P = sinkhorn.Problem([rng.uniform(0, 1, (5, 6))], 0.5, 0.0, 0.5, 2)
    sol = sinkhorn.solve(P, 1e7, tol=1e-13, n_max=1000)
    Q = sinkhorn.plan_blocks(P, sol["f"], sol["g"], 1e7)[0]
    # eps -> infinity: the product plan a b^T / (|I| + T_b), whatever the costs
    assert np.allclose(Q, 1.0 / (5 + P.t_b), rtol=1e-5)


def test_dual_is_non_decreasing():
    rng = np.random.default_rng(3)
    P = _problem(rng, [(6, 5), (4, 4), (8, 6)])
    sol = sinkhorn.solve(P, 0.3, tol=1e-14, n_max=300, history=True)
    d = np.array(sol["dual"])
    assert np.all(np.diff(d) >= -1e-10 * np.abs(d[1:]))


def _lp_plan(P):
    """Exact eps -> 0 plan by expanding row 0 into T_b copies and column 0 into
    T_a copies: a square assignment problem of size |I| + T_b."""
    I, J, tb, ta = P.I, P.J, int(P.t_b), int(P.t_a)
    n = I + tb
    assert J + ta == n
    big = 1e9
    M = np.full((n, n), big)
    for b, C in enumerate(P.C):
        r0, c0 = P.row_off[b], P.col_off[b]
        M[r0:r0 + C.shape[0], c0:c0 + C.shape[1]] = C
    M[:I, J:] = P.c_out
    M[I:, :J] = P.c_unm
    M[I:, J:] = P.c_sink
    return M


def _brute(M):
    n = M.shape[0]
    best, arg = np.inf, None
    for perm in itertools.permutations(range(n)):
        v = M[np.arange(n), perm].sum()
        if v < best - 1e-12:
            best, arg = v, perm
    return best, arg


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_eps_to_zero_matches_assignment(seed):
    rng = np.random.default_rng(seed)
    P = sinkhorn.Problem([rng.uniform(0, 4, (3, 2)), rng.uniform(0, 4, (2, 2))], 2.5, 0.0, 2.5, 1)
    M = _lp_plan(P)
    best, perm = _brute(M)
    r, c = linear_sum_assignment(M)
    assert M[r, c].sum() == pytest.approx(best)
    eps = 2e-3
    f = g = None
    f0 = g0 = 0.0
    for e in np.geomspace(1.0, eps, 12):        # eps-scaling warm starts
        sol = sinkhorn.solve(P, e, tol=1e-10, n_max=20000, f=f, g=g, f0=f0, g0=g0)
        f, g, f0, g0 = sol["f"], sol["g"], sol["f0"], sol["g0"]
    assert sol["err"] <= 1e-10
    Qb = sinkhorn.plan_blocks(P, sol["f"], sol["g"], eps)
    # LP plan on the I x J part
    Z = np.zeros((P.I, P.J))
    for i in range(P.I):
        if perm[i] < P.J:
            Z[i, perm[i]] = 1.0
    Qf = np.zeros((P.I, P.J))
    for b, q in enumerate(Qb):
        Qf[P.row_off[b]:P.row_off[b + 1], P.col_off[b]:P.col_off[b + 1]] = q
    assert np.max(np.abs(Qf - Z)) < 1e-3
    # and the minimal matched count is |J| - T_b
    assert Z.sum() == P.J - P.t_b


def test_infeasible_masses_rejected():
    with pytest.raises(ValueError):
        sinkhorn.Problem([np.zeros((1, 5))], 1.0, 0.0, 1.0, 1)


def test_hard_assignment_and_objectives():
    rng = np.random.default_rng(7)
    P = _problem(rng, [(5, 4), (3, 3)], c_out=0.5, spread=5.0)
    sol = sinkhorn.solve(P, 0.05, tol=1e-10, n_max=50000)
    js, qs, qi0 = sinkhorn.hard_assignment(P, sol["f"], sol["g"], sol["f0"], sol["g0"], 0.05)
    assert np.all(qs >= qi0 - 1e-15)
    ob = sinkhorn.objectives(P, sol["f"], sol["g"], sol["f0"], sol["g0"], 0.05, 1.0, 150.0)
    assert ob["mass"] == pytest.approx(P.I + P.t_b, rel=1e-10)
    assert ob["entropy"] >= 0
