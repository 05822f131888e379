"""Pins of the oracle M-step: finite differences, quadratic convergence,
agreement with the paper's Newton + MM route, Wahba, and EM exact recovery."""
import numpy as np
import pytest

import inputgen as ig
from oracle import cost, crystal, em, forward, metrics, mstep, simulate, sinkhorn

D = 150.0


def _pairs(seed=0, noise=0.3, n_rot=6):
    p = ig.MEDIUM
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry(n_rot, np.deg2rad(30.0), p.detectors, p.lam_min, p.lam_max)
    rng = np.random.default_rng(seed)
    q = ig.random_quaternions(rng, 1)
    x = ig.random_positions(rng, 1, 2.5, 5.0)
    S = forward.enumerate_visible(pl, q, x, g)
    K = len(S["m"])
    # detected spot = model spot moved in the detector plane; several weights per model spot
    p_lab = np.repeat(S["s"], 2, axis=0)
    p_lab[:, 1:] += rng.normal(0, noise, (2 * K, 2))
    t = np.repeat(S["t"], 2)
    w = np.repeat(pl["w"][S["m"]], 2, axis=0)
    wt = rng.uniform(0.2, 1.0, 2 * K)
    return mstep.Pairs(p_lab, t, w, wt), q[0], x[0], g


def test_jacobian_finite_differences():
    pairs, q, x, g = _pairs()
    R = crystal.quat_to_R(q)
    rho, J = mstep.residuals_jacobians(pairs, R, x, g, D)
    h = 1e-6
    for k in range(6):
        dth = np.zeros(6)
        dth[k] = h
        qa, xa = mstep.apply_step(q, x, dth[:3], dth[3:])
        qb, xb = mstep.apply_step(q, x, -dth[:3], -dth[3:])
        ra, _ = mstep.residuals_jacobians(pairs, crystal.quat_to_R(qa), xa, g, D)
        rb, _ = mstep.residuals_jacobians(pairs, crystal.quat_to_R(qb), xb, g, D)
        num = (ra - rb) / (2 * h)
        assert np.allclose(J[:, :, k], num, rtol=1e-6, atol=1e-6 * np.abs(num).max())


def test_gradient_matches_objective_derivative():
    pairs, q, x, g = _pairs(seed=1)
    R = crystal.quat_to_R(q)
    H, grad = mstep.normal_equations(pairs, R, x, g, D)
    h = 1e-6
    for k in range(6):
        dth = np.zeros(6)
        dth[k] = h
        qa, xa = mstep.apply_step(q, x, dth[:3], dth[3:])
        qb, xb = mstep.apply_step(q, x, -dth[:3], -dth[3:])
        fa = mstep.objective(pairs, crystal.quat_to_R(qa), xa, g, D)
        fb = mstep.objective(pairs, crystal.quat_to_R(qb), xb, g, D)
        assert (fa - fb) / (2 * h) == pytest.approx(2 * grad[k], rel=1e-6, abs=1e-6)
    assert np.allclose(H, H.T)
    assert np.all(np.linalg.eigvalsh(H) > 0)


def test_zero_residual_converges_quadratically():
    pairs, q, x, g = _pairs(seed=2, noise=0.0)
    q1, x1 = ig.perturb_grains(q[None], x[None], 0.3, 0.3, 5)
    q1, x1 = q1[0], x1[0]
    errs = []
    for _ in range(5):
        q1, x1, st, _, _, _ = mstep.gn_step(pairs, q1, x1, g, D)
        errs.append(np.degrees(metrics.misorientation(q1, q)) + np.linalg.norm(x1 - x))
    assert errs[3] < 1e-9
    assert errs[1] < 1e-2 * errs[0] ** 1.5 + 1e-12
    R = crystal.quat_to_R(q1)
    assert np.allclose(R.T @ R, np.eye(3), atol=1e-12) and np.linalg.det(R) == pytest.approx(1.0)


def test_gn_and_paper_newton_mm_reach_same_point():
    pairs, q, x, g = _pairs(seed=3, noise=0.4)
    qg, xg = q.copy(), x.copy()
    for _ in range(30):
        qg, xg, _, _, _, _ = mstep.gn_step(pairs, qg, xg, g, D)
    # coordinate descent: LauePosNewton on x, LaueRotMM on R, alternated
    R, xc = crystal.quat_to_R(q), x.copy()
    for _ in range(60):
        xc = mstep.pos_newton(pairs, R, xc, g)
        R = mstep.rot_mm(pairs, R, xc, g)
    assert np.allclose(xc, xg, atol=1e-7)
    assert np.degrees(metrics.misorientation(crystal.R_to_quat(R), qg)) < 1e-7


def test_rot_mm_is_monotone():
    pairs, q, x, g = _pairs(seed=4, noise=0.5)
    R = crystal.quat_to_R(ig.perturb_grains(q[None], x[None], 1.0, 0.0, 3)[0][0])
    vals = [mstep.mm_objective(pairs, R, x, g)]
    for _ in range(6):
        R = mstep.rot_mm(pairs, R, x, g, n_iter=1)
        vals.append(mstep.mm_objective(pairs, R, x, g))
    assert np.all(np.diff(vals) >= -1e-12)


def test_wahba():
    rng = np.random.default_rng(8)
    Rt = crystal.quat_to_R(ig.random_quaternions(rng, 1))[0]
    b = rng.standard_normal((5, 3))
    a = b @ Rt.T
    assert np.allclose(mstep.wahba(a, b, np.ones(5)), Rt, atol=1e-12)
    # a reflected target still yields a proper rotation
    Rr = mstep.wahba(b * [1, 1, -1], b, np.ones(5))
    assert np.linalg.det(Rr) == pytest.approx(1.0)


def test_em_noise_free_exact_recovery():
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
                 cost.c_out(p.sigma_mm, p.distance), t_b=sinkhorn.default_tb(len(model["m"]), 0.1))
    assert np.max(np.degrees(metrics.misorientation(res["q"], q))) < 1e-6
    assert np.max(np.linalg.norm(res["x"] - x, axis=1)) < 1e-6


def test_pos_grad_hess_finite_differences():
    """Eqs. xgrad and xhess (with the chain rule through y = Gamma_t x) against
    central differences of F(x) = sum Q rhat^T r."""
    pairs, q, x, g = _pairs(seed=5, noise=0.4)
    R = crystal.quat_to_R(q)
    gx, Hx = mstep.pos_grad_hess(pairs, R, x, g)
    h = 1e-4
    for k in range(3):
        dx = np.zeros(3)
        dx[k] = h
        fa = mstep.mm_objective(pairs, R, x + dx, g)
        fb = mstep.mm_objective(pairs, R, x - dx, g)
        assert (fa - fb) / (2 * h) == pytest.approx(gx[k], rel=1e-6, abs=1e-9)
        ga, _ = mstep.pos_grad_hess(pairs, R, x + dx, g)
        gb, _ = mstep.pos_grad_hess(pairs, R, x - dx, g)
        assert np.allclose((ga - gb) / (2 * h), Hx[:, k], rtol=1e-5, atol=1e-9 * np.abs(Hx).max())
    assert np.allclose(Hx, Hx.T)


def test_m0_matrices_give_the_objective():
    """Eq. qcoc: sum_m w_m^T R^T M0_m R w_m differs from F(R) = sum Q rhat^T r
    by a constant, for any two rotations."""
    pairs, q, x, g = _pairs(seed=6, noise=0.4)
    _, W, M0 = mstep.m0_matrices(pairs, x, g)
    rng = np.random.default_rng(1)
    Rs = crystal.quat_to_R(ig.random_quaternions(rng, 3))
    G = [float(np.einsum("ma,mab,mb->", W @ R.T, M0, W @ R.T)) for R in Rs]
    F = [mstep.mm_objective(pairs, R, x, g) for R in Rs]
    for k in (1, 2):
        assert G[k] - G[0] == pytest.approx(F[k] - F[0], rel=1e-10, abs=1e-9)


def test_m0_per_plane_index_keeps_harmonics_apart():
    """Eq. M0 sums over the model spots of one plane m: two planes with the
    same normal (a harmonic pair) keep their own matrices (and shifts)."""
    pairs, q, x, g = _pairs(seed=7)
    K = len(pairs.q)
    m = np.arange(K) % 2                     # two plane ids over pairs that share no normal structure
    pairs.w[:] = pairs.w[0]                  # one normal for every pair
    keyed = mstep.Pairs(pairs.p, pairs.t, pairs.w, pairs.q, m)
    keys, W, M0 = mstep.m0_matrices(keyed, x, g)
    assert sorted(keys) == [0, 1] and len(M0) == 2
    _, _, M0w = mstep.m0_matrices(pairs, x, g)
    assert len(M0w) == 1 and np.allclose(M0[0] + M0[1], M0w[0])


def test_mm_shift_is_psd_and_minimal():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((3, 3))
    M0 = -(A @ A.T) + 0.1 * np.eye(3)
    M = mstep.mm_shift(M0)
    ev = np.linalg.eigvalsh(M)
    assert ev[0] == pytest.approx(0.0, abs=1e-12) and np.all(ev >= -1e-12)
    P = A @ A.T
    assert np.array_equal(mstep.mm_shift(P), P)


def test_paper_step_stationary_point_and_em_recovery():
    """A sweep from the GN optimum stays there; the EM with the paper's
    M-step recovers noise-free grains exactly (four sweeps per EM iteration:
    coordinate descent between x and R converges linearly)."""
    pairs, q, x, g = _pairs(seed=3, noise=0.4)
    qg, xg = q.copy(), x.copy()
    for _ in range(30):
        qg, xg, _, _, _, _ = mstep.gn_step(pairs, qg, xg, g, D)
    qp, xp = mstep.paper_step(pairs, qg, xg, g)
    assert np.degrees(metrics.misorientation(qp, qg)) < 1e-7 and np.allclose(xp, xg, atol=1e-8)
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    geo = forward.Geometry.from_preset(p)
    qt, xt = ig.random_grains(p)
    sim = simulate.simulate(pl, qt, xt, geo, 0.0, 0.0, p.seed, p.distance)
    q0, x0 = ig.perturb_grains(qt, xt, 0.5, 0.5, 1)
    model = forward.enumerate_visible(pl, q0, x0, geo)
    model["offsets"] = forward.block_offsets(model["block"], geo.n_blocks)
    eps = em.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    res = em.run(pl, geo, p.distance, sim["p12"], sim["offsets"], model, q0, x0, eps,
                 cost.c_out(p.sigma_mm, p.distance), k_gn=4, mstep_method="paper",
                 paper_kw={"n_newton": 4, "tol_x": 1e-12, "n_mm": 500, "tol_r": 1e-13})
    assert np.max(np.degrees(metrics.misorientation(res["q"], qt))) < 1e-6
    assert np.max(np.linalg.norm(res["x"] - xt, axis=1)) < 1e-6
