"""Pins of the sparse (rho nearest neighbours) oracle against what the paper
and the mathematics fix: the neighbour sets by brute force, the dense
problem when every column is a neighbour, null weight outside the sets, the
error bound of the approximation, and noise-free EM recovery."""
import itertools
import math

import numpy as np
import pytest

import inputgen as ig
from oracle import cost, crystal, em, forward, metrics, simulate, sinkhorn, sparse


def _blocks(rng, shapes):
    return [rng.uniform(0.0, 50.0, s) for s in shapes]


@pytest.mark.parametrize("rho", [1, 3, 7, 40])
def test_neighbour_sets_brute_force(rho):
    rng = np.random.default_rng(rho)
    C = rng.uniform(0.0, 10.0, (9, 12))
    C[:, 5] = C[:, 2]          # exact ties between columns 2 and 5
    C[3, :] = 1.0              # a row of all-equal costs
    nb = sparse.neighbours(C, rho)
    k = min(rho, C.shape[1])
    assert nb.shape == (9, k)
    for i in range(C.shape[0]):
        kept = set(nb[i].tolist())
        assert len(kept) == k
        # every kept cost <= every dropped cost; on equal costs the lower index is kept
        for a, b in itertools.product(kept, set(range(C.shape[1])) - kept):
            assert C[i, a] < C[i, b] or (C[i, a] == C[i, b] and a < b)
        # ordered by (cost, index)
        assert all((C[i, nb[i, t]], nb[i, t]) < (C[i, nb[i, t + 1]], nb[i, t + 1]) for t in range(k - 1))
    assert sorted(nb[3].tolist()) == list(range(k))


def test_empty_blocks():
    assert sparse.neighbours(np.zeros((4, 0)), 8).shape == (4, 0)
    assert sparse.neighbours(np.zeros((0, 5)), 8).shape == (0, 5)
    M = sparse.masked_blocks([np.zeros((0, 3)), np.zeros((2, 0))], 2)
    assert M[0].shape == (0, 3) and M[1].shape == (2, 0)


def test_all_neighbours_is_the_dense_problem():
    rng = np.random.default_rng(1)
    C = _blocks(rng, [(6, 5), (4, 7), (3, 2)])
    P = sinkhorn.Problem(C, 9.0, 0.0, 9.0, 4.0)
    S = sparse.masked_problem(P, 7)
    for a, b in zip(P.C, S.C):
        assert np.array_equal(a, b)
    d = sinkhorn.solve(P, 5.0, tol=1e-12, n_max=5000)
    s = sinkhorn.solve(S, 5.0, tol=1e-12, n_max=5000)
    assert np.array_equal(d["f"], s["f"]) and np.array_equal(d["g"], s["g"])


def test_null_weight_outside_and_marginals():
    rng = np.random.default_rng(2)
    C = _blocks(rng, [(20, 15), (12, 18)])
    P = sparse.masked_problem(sinkhorn.Problem(C, 30.0, 0.0, 30.0, 10.0), 3)
    sol = sinkhorn.solve(P, 4.0, tol=1e-12, n_max=20000)
    Qb = sinkhorn.plan_blocks(P, sol["f"], sol["g"], 4.0)
    for Q, Cb, Mb in zip(Qb, C, P.C):
        nb = sparse.neighbours(Cb, 3)
        mask = np.zeros(Cb.shape, bool)
        mask[np.repeat(np.arange(Cb.shape[0]), 3), nb.ravel()] = True
        assert np.all(Q[~mask] == 0.0)
        assert np.all(Q[mask] > 0.0)
    rows, row0, cols, col0 = sinkhorn.marginals(P, sol["f"], sol["g"], sol["f0"], sol["g0"], 4.0)
    assert np.allclose(rows, 1.0, atol=1e-10) and np.allclose(cols, 1.0, atol=1e-10)
    assert row0 == pytest.approx(P.t_b, rel=1e-10) and col0 == pytest.approx(P.t_a, rel=1e-10)


def test_approximation_error_bound():
    """Each detected spot has one model spot at cost ~0 and the rest >= Delta:
    the sparse plan differs from the dense one by no more than a small
    multiple of the mass the dense plan puts outside the neighbour sets."""
    rng = np.random.default_rng(3)
    n = 10
    C = 40.0 + rng.uniform(0.0, 5.0, (n, n))
    C[np.arange(n), rng.permutation(n)] = rng.uniform(0.0, 0.5, n)
    eps = 1.5
    P = sinkhorn.Problem([C], 20.0, 0.0, 20.0, 2.0)
    S = sparse.masked_problem(P, 1)
    d = sinkhorn.solve(P, eps, tol=1e-13, n_max=20000)
    s = sinkhorn.solve(S, eps, tol=1e-13, n_max=20000)
    Qd = sinkhorn.plan_blocks(P, d["f"], d["g"], eps)[0]
    Qs = sinkhorn.plan_blocks(S, s["f"], s["g"], eps)[0]
    kept = np.zeros(C.shape, bool)
    kept[np.arange(n), sparse.neighbours(C, 1)[:, 0]] = True
    dropped = float(Qd[~kept].sum())
    assert 0.0 < dropped < 1e-9
    assert np.max(np.abs(Qd - Qs)) <= 4.0 * dropped + 1e-15


def test_eps_init_closed_form():
    C = [np.array([[1.0, 2.0, 9.0], [4.0, 0.5, 3.0], [7.0, 7.5, 0.0]])]
    # farthest of the 2 nearest: rows -> 2.0, 3.0, 7.0; median 3.0
    assert sparse.farthest_costs(C, 2).tolist() == [2.0, 3.0, 7.0]
    assert sparse.eps_init(C, 2) == pytest.approx(3.0 / math.log(100.0))


def test_sparse_em_noise_free_exact_recovery():
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry.from_preset(p)
    q, x = ig.random_grains(p)
    sim = simulate.simulate(pl, q, x, g, 0.0, 0.0, p.seed, p.distance)
    q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, 1)
    model = forward.enumerate_visible(pl, q0, x0, g)
    model["offsets"] = forward.block_offsets(model["block"], g.n_blocks)
    eps = em.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    res = em.run(pl, g, p.distance, sim["p12"], sim["offsets"], model, q0, x0, eps,
                 cost.c_out(p.sigma_mm, p.distance), t_b=sinkhorn.default_tb(len(model["m"]), 0.1), rho=4)
    assert np.max(np.degrees(metrics.misorientation(res["q"], q))) < 1e-6
    assert np.max(np.linalg.norm(res["x"] - x, axis=1)) < 1e-6


def test_objectives_count_kept_entries_only():
    """The plan summaries of a masked problem sum over the kept entries (and
    the bins) only: the masked entries' 0 * inf terms are 0."""
    rng = np.random.default_rng(7)
    C = _blocks(rng, [(6, 7), (4, 3)])
    P = sparse.masked_problem(sinkhorn.Problem(C, 9.0, 0.0, 9.0, 2.0), 2)
    s = sinkhorn.solve(P, 1.5, tol=1e-10, n_max=10000)
    o = sinkhorn.objectives(P, s["f"], s["g"], s["f0"], s["g0"], 1.5)
    Q = sinkhorn.plan_blocks(P, s["f"], s["g"], 1.5)
    inl = 0.0
    for q, Cd, Cm in zip(Q, C, P.C):
        kept = np.isfinite(Cm)
        inl += float(np.sum(q[kept] * Cd[kept]))
        assert np.all(q[~kept] == 0.0)
    assert np.isfinite(o["cost_inlier"]) and o["cost_inlier"] == pytest.approx(inl, rel=1e-12)
    assert np.isfinite(o["entropy"]) and o["mass"] == pytest.approx(P.I + P.t_b, rel=1e-9)
