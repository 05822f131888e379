"""Pins of the unbalanced-OT oracle against what the paper's Problem B and the
mathematics fix: the one-entry closed form, optimality of the primal at the
computed plan, the first-order marginal conditions (which tell kappa's side
from lambda's), the contraction rate of the iteration, the balanced limit
(an optimal assignment by a library solver), masked entries, empty rows and
columns, and the hard assignment on a hand-worked case."""
import math

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import unbalanced as ub


def _blocks(rng, shapes, hi=8.0):
    return [rng.uniform(0.0, hi, s) for s in shapes]


@pytest.mark.parametrize("c,eps,kappa,lam", [(3.0, 1.0, 0.5, 2.0), (0.2, 0.05, 1.0, 1.0), (7.0, 2.0, 0.1, 0.3)])
def test_single_entry_closed_form(c, eps, kappa, lam):
    """One detected and one model spot: d/dq [q c + eps (q log q - q) +
    (kappa + lambda)(q log q - q + 1)] = 0 gives q = exp(-c / (eps + kappa + lambda))."""
    sol = ub.solve([np.array([[c]])], eps, kappa, lam, tol=1e-14, n_max=100000)
    q = ub.plan_blocks([np.array([[c]])], sol["f"], sol["g"], eps)[0][0, 0]
    assert q == pytest.approx(math.exp(-c / (eps + kappa + lam)), rel=1e-10)


@pytest.mark.parametrize("kappa,lam", [(0.3, 3.0), (3.0, 0.3), (1.0, 1.0)])
def test_first_order_marginals(kappa, lam):
    """At the optimum of Problem B, row_i = exp(-f_i / kappa) and
    col_j = exp(-g_j / lambda): kappa belongs to the detected-spot side."""
    rng = np.random.default_rng(5)
    C = _blocks(rng, [(7, 5), (4, 9), (6, 6)])
    eps = 0.7
    sol = ub.solve(C, eps, kappa, lam, tol=1e-14, n_max=100000)
    rows, cols = ub.marginals(C, sol["f"], sol["g"], eps)
    assert np.allclose(rows, np.exp(-sol["f"] / kappa), rtol=1e-10, atol=1e-14)
    assert np.allclose(cols, np.exp(-sol["g"] / lam), rtol=1e-10, atol=1e-14)


def test_primal_optimality_under_perturbation():
    """The computed plan minimises Problem B's primal: every multiplicative
    perturbation of it, in random directions, costs more."""
    rng = np.random.default_rng(6)
    C = _blocks(rng, [(6, 4), (3, 5)])
    eps, kappa, lam = 0.8, 0.4, 1.7
    sol = ub.solve(C, eps, kappa, lam, tol=1e-14, n_max=100000)
    Q = ub.plan_blocks(C, sol["f"], sol["g"], eps)
    p0 = ub.primal(C, Q, eps, kappa, lam)
    for t in range(40):
        step = 10.0 ** rng.uniform(-4, -1)
        Qp = [q * np.exp(step * rng.standard_normal(q.shape)) for q in Q]
        assert ub.primal(C, Qp, eps, kappa, lam) > p0
    # the plan with the two exponents swapped is not optimal when kappa != lambda
    sw = ub.solve(C, eps, lam, kappa, tol=1e-14, n_max=100000)
    assert ub.primal(C, ub.plan_blocks(C, sw["f"], sw["g"], eps), eps, kappa, lam) > p0 + 1e-6


def test_contraction_rate():
    """Each half is a tau-contraction of the potentials in the max norm (LSE
    is 1-Lipschitz), so successive changes fall at least by tau_r tau_c."""
    rng = np.random.default_rng(7)
    C = _blocks(rng, [(10, 8), (5, 12)])
    eps, kappa, lam = 1.0, 2.0, 0.5
    tau = kappa / (kappa + eps) * lam / (lam + eps)
    errs = []
    f, g = np.zeros(sum(c.shape[0] for c in C)), np.zeros(sum(c.shape[1] for c in C))
    for _ in range(12):
        s = ub.solve(C, eps, kappa, lam, tol=0.0, n_max=1, f=f, g=g)
        errs.append(max(np.max(np.abs(s["f"] - f)), np.max(np.abs(s["g"] - g))))
        f, g = s["f"], s["g"]
    for a, b in zip(errs[1:], errs[2:]):
        assert b <= tau * a * (1 + 1e-9) + 1e-15


def test_stopping_value_is_the_marginal_change():
    """The stopping value is the largest change an update makes to a plan
    marginal: a row half from (f, g) moves row i from S_i to
    S_i exp((f'_i - f_i)/eps), checked against plan sums taken directly."""
    rng = np.random.default_rng(10)
    C = _blocks(rng, [(5, 7), (6, 4)])
    eps, kappa, lam = 0.9, 0.7, 1.3
    f, g = rng.normal(0, 0.5, 11), rng.normal(0, 0.5, 11)
    s = ub.solve(C, eps, kappa, lam, tol=0.0, n_max=1, f=f, g=g)
    r0 = ub.marginals(C, f, g, eps)[0]
    r1 = ub.marginals(C, s["f"], g, eps)[0]
    c0 = ub.marginals(C, s["f"], g, eps)[1]
    c1 = ub.marginals(C, s["f"], s["g"], eps)[1]
    want = max(np.max(np.abs(r1 - r0)), np.max(np.abs(c1 - c0)))
    assert s["err"] == pytest.approx(want, rel=1e-12)
    # a row far from everything moves its potential a lot but its (zero) mass not at all
    Cf = [np.vstack([C[0], np.full((1, 7), 1e4)]), C[1]]
    s = ub.solve(Cf, eps, kappa, lam, tol=1e-9, n_max=10000)
    assert s["err"] <= 1e-9 and s["f"][5] > 1e3


def test_balanced_limit_is_an_optimal_assignment():
    """kappa, lambda >> costs and small eps: the plan concentrates on a
    minimum-cost perfect matching (square block, separated optimum)."""
    rng = np.random.default_rng(8)
    n = 6
    C = rng.uniform(2.0, 6.0, (n, n))
    perm = rng.permutation(n)
    C[np.arange(n), perm] = rng.uniform(0.0, 0.3, n)
    r, c = linear_sum_assignment(C)
    sol = ub.solve([C], 0.05, 200.0, 200.0, tol=1e-11, n_max=100000)
    Q = ub.plan_blocks([C], sol["f"], sol["g"], 0.05)[0]
    P = np.zeros_like(C)
    P[r, c] = 1.0
    # matched mass falls short of 1 by about c / (kappa + lambda) <= 1e-3
    assert np.max(np.abs(Q - P)) < 2e-3


def test_masked_entries_and_empty_sides():
    rng = np.random.default_rng(9)
    C = _blocks(rng, [(5, 6), (3, 0), (0, 4), (4, 3)])
    C[0][1, :] = np.inf              # a row with no kept entry
    C[0][:, 2] = np.inf              # a column with no kept entry
    C[3][0, 1] = np.inf
    eps, kappa, lam = 0.9, 1.1, 0.6
    sol = ub.solve(C, eps, kappa, lam, tol=1e-13, n_max=100000)
    f, g = sol["f"], sol["g"]
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(g))
    assert f[1] == 0.0 and g[2] == 0.0
    assert np.all(f[5:8] == 0.0)              # rows of the block without model spots
    assert np.all(g[6:10] == 0.0)             # columns of the block without detected spots
    Q = ub.plan_blocks(C, f, g, eps)
    assert np.all(Q[0][1] == 0.0) and np.all(Q[0][:, 2] == 0.0) and Q[3][0, 1] == 0.0
    rows, cols = ub.marginals(C, f, g, eps)
    live_r = rows > 0
    live_c = cols > 0
    assert np.allclose(rows[live_r], np.exp(-f[live_r] / kappa), rtol=1e-10)
    assert np.allclose(cols[live_c], np.exp(-g[live_c] / lam), rtol=1e-10)


def test_hard_assignment_hand_worked():
    """Potentials set by hand: row 0 puts 0.7 on column 1 (deficit 0.2 <
    0.7: assigned), row 1 puts 0.1 + 0.1 (deficit 0.8: outlier), row 2 has
    equal entries 0.45 (deficit 0.1: lowest index)."""
    eps = 1.0
    C = np.array([[-math.log(0.1), -math.log(0.7)],
                  [-math.log(0.1), -math.log(0.1)],
                  [-math.log(0.45), -math.log(0.45)]])
    js, qs, qo = ub.hard_assignment([C], np.zeros(3), np.zeros(2), eps)
    assert js.tolist() == [1, -1, 0]
    assert qs == pytest.approx([0.7, 0.8, 0.45])
    assert qo == pytest.approx([0.2, 0.8, 0.1])


@pytest.mark.parametrize("rho", [None, 4])
def test_unbalanced_em_noise_free_exact_recovery(rho):
    import inputgen as ig
    from oracle import cost, crystal, em, forward, metrics, simulate
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry.from_preset(p)
    q, x = ig.random_grains(p)
    sim = simulate.simulate(pl, q, x, g, 0.0, 0.0, p.seed, p.distance)
    q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, 1)
    model = forward.enumerate_visible(pl, q0, x0, g)
    model["offsets"] = forward.block_offsets(model["block"], g.n_blocks)
    eps = em.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    s2 = 2.0 * p.sigma_mm ** 2
    res = em.run(pl, g, p.distance, sim["p12"], sim["offsets"], model, q0, x0, eps,
                 cost.c_out(p.sigma_mm, p.distance), rho=rho, unbalanced_kl=(0.5 * s2, 0.5 * s2))
    assert res["f0"] == -np.inf and res["g0"] == -np.inf
    assert np.max(np.degrees(metrics.misorientation(res["q"], q))) < 1e-6
    assert np.max(np.linalg.norm(res["x"] - x, axis=1)) < 1e-6
