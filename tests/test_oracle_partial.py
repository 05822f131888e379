"""Pins of the partial-OT oracle against what the paper's Problem A and the
mathematics fix: the potential iteration equals Dykstra's projections on
dense matrices step by step, the result equals a generic constrained
solver's, the first-order (KKT) conditions, the full-mass limit, masked
entries and empty sides, and noise-free EM recovery."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import partial as po


def _blocks(rng, shapes, hi=6.0):
    return [rng.uniform(0.0, hi, s) for s in shapes]


@pytest.mark.parametrize("n_iter", [1, 2, 5, 40])
def test_potential_form_equals_dykstra(n_iter):
    rng = np.random.default_rng(n_iter)
    C = rng.uniform(0.0, 4.0, (6, 8))
    eps, frac = 0.7, 0.6
    sol = po.solve([C], eps, frac, tol=0.0, n_max=n_iter)
    Q = po.plan_blocks([C], sol["f"], sol["g"], eps)[0]
    D = po.dykstra(C, eps, frac * 6, n_iter)
    assert np.allclose(Q, D, rtol=1e-10, atol=1e-14)


def test_matches_a_generic_constrained_solver():
    rng = np.random.default_rng(3)
    C = rng.uniform(0.0, 3.0, (3, 4))
    eps, frac = 0.8, 0.7
    m = frac * 3
    sol = po.solve([C], eps, frac, tol=1e-13, n_max=100000)
    Q = po.plan_blocks([C], sol["f"], sol["g"], eps)[0]

    def obj(q):
        q = np.maximum(q, 1e-300)
        return float(np.sum(q * C.ravel()) + eps * np.sum(q * (np.log(q) - 1.0)))

    def grad(q):
        return C.ravel() + eps * np.log(np.maximum(q, 1e-300))
    cons = [{"type": "eq", "fun": lambda q: q.sum() - m},
            {"type": "ineq", "fun": lambda q: 1.0 - q.reshape(3, 4).sum(axis=1)},
            {"type": "ineq", "fun": lambda q: 1.0 - q.reshape(3, 4).sum(axis=0)}]
    r = minimize(obj, np.full(12, m / 12), jac=grad, bounds=[(1e-12, 1.0)] * 12, constraints=cons,
                 method="SLSQP", options={"ftol": 1e-15, "maxiter": 2000})
    assert r.success
    assert np.max(np.abs(r.x.reshape(3, 4) - Q)) < 1e-5
    assert obj(Q.ravel()) <= r.fun + 1e-9


def test_first_order_conditions():
    """Q = exp((f' + g' + h - c)/eps) with f', g' <= 0, a saturated row (column)
    wherever its potential is negative, rows and columns <= 1, mass m."""
    rng = np.random.default_rng(4)
    C = _blocks(rng, [(7, 5), (4, 9), (6, 6)])
    eps, frac = 0.5, 0.8
    sol = po.solve(C, eps, frac, tol=1e-13, n_max=100000)
    fp = sol["f"] - sol["h"]
    g = sol["g"]
    rows, cols = po.marginals(C, sol["f"], g, eps)
    assert np.all(fp <= 1e-12) and np.all(g <= 1e-12)
    assert np.all(rows <= 1 + 1e-9) and np.all(cols <= 1 + 1e-9)
    assert rows.sum() == pytest.approx(sol["mass"], rel=1e-10)
    assert sol["mass"] == pytest.approx(frac * (5 + 4 + 6))
    assert np.all(np.abs(rows[fp < -1e-6] - 1) < 1e-8)
    assert np.all(np.abs(cols[g < -1e-6] - 1) < 1e-8)
    # some rows are saturated and some are not at this mass
    assert (fp < -1e-6).any() and (fp > -1e-9).any()


def test_full_mass_square_block_is_balanced():
    rng = np.random.default_rng(5)
    C = rng.uniform(0.0, 3.0, (5, 5))
    sol = po.solve([C], 0.6, 1.0, tol=1e-12, n_max=200000)
    rows, cols = po.marginals([C], sol["f"], sol["g"], 0.6)
    assert np.allclose(rows, 1.0, atol=1e-9) and np.allclose(cols, 1.0, atol=1e-9)


def test_masked_entries_empty_sides_and_stop():
    rng = np.random.default_rng(6)
    C = _blocks(rng, [(5, 6), (3, 0), (0, 4), (4, 3)])
    C[0][1, :] = np.inf
    C[0][:, 2] = np.inf
    sol = po.solve(C, 0.9, 0.5, tol=1e-10, n_max=100000, history=True)
    f, g = sol["f"], sol["g"]
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(g))
    assert g[2] == 0.0 and np.all(g[6:10] == 0.0)
    Q = po.plan_blocks(C, f, g, 0.9)
    assert np.all(Q[0][1] == 0.0) and np.all(Q[0][:, 2] == 0.0)
    assert sum(q.sum() for q in Q) == pytest.approx(sol["mass"], rel=1e-9)
    errs = sol["errs"]
    assert np.isinf(errs[0]) and errs[-1] <= 1e-10 and sol["n_iter"] == len(errs)


def test_partial_em_noise_free_exact_recovery():
    import inputgen as ig
    from oracle import cost, crystal, em, forward, metrics, simulate
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    geo = forward.Geometry.from_preset(p)
    q, x = ig.random_grains(p)
    sim = simulate.simulate(pl, q, x, geo, 0.0, 0.0, p.seed, p.distance)
    q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, 1)
    model = forward.enumerate_visible(pl, q0, x0, geo)
    model["offsets"] = forward.block_offsets(model["block"], geo.n_blocks)
    eps = em.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    res = em.run(pl, geo, p.distance, sim["p12"], sim["offsets"], model, q0, x0, eps,
                 cost.c_out(p.sigma_mm, p.distance), partial_frac=0.9)
    assert res["f0"] == -np.inf
    assert np.max(np.degrees(metrics.misorientation(res["q"], q))) < 1e-6
    assert np.max(np.linalg.norm(res["x"] - x, axis=1)) < 1e-6
