"""Pins of oracle parts whose values are otherwise checked only against
themselves: the plan summaries (Eqs. elbo, estep_obj), the pair features of
the spot-pair candidates, the SPOT values of the single-grain score (App. E)
and the paper's annealing modes (Sec. 5.1, Sec. 7, App. D, Alg. LaueOT)."""
import math

import numpy as np
import pytest

import inputgen as ig
from oracle import candidates, cost, crystal, em, forward, metrics, simulate, single, sinkhorn, sparse

D = 150.0
A_BCC = 2.87


def _rand_problem(rng, sizes, c_out=2.0, t_b=None, spread=3.0):
    C = [rng.uniform(0, spread, s) for s in sizes]
    J = sum(s[1] for s in sizes)
    return sinkhorn.Problem(C, c_out, 0.0, c_out, math.ceil(0.4 * J) if t_b is None else t_b)


# ---------------------------------------------------------------- plan summaries

@pytest.mark.parametrize("seed,eps", [(0, 0.7), (1, 0.2), (2, 3.0)])
def test_objectives_entropic_duality_at_convergence(seed, eps):
    """With log Q = (f + g - c)/eps every entry satisfies c Q - eps (-Q log Q) =
    (f_i + g_j) Q, so at the marginals (1 per spot, T_b for row 0, T_a for
    column 0) the total cost minus eps times the entropy equals the dual sum
    sum_i f_i + sum_j g_j + T_b f_0 + T_a g_0.  A dropped bin term, a wrong
    sign of the entropy or a missing 1/eps fails this."""
    rng = np.random.default_rng(seed)
    P = _rand_problem(rng, [(5, 4), (3, 6), (0, 2), (4, 0), (6, 5)])
    sol = sinkhorn.solve(P, eps, tol=1e-13, n_max=200000)
    f, g, f0, g0 = sol["f"], sol["g"], sol["f0"], sol["g0"]
    ob = sinkhorn.objectives(P, f, g, f0, g0, eps, 1.0, D)
    dual = f.sum() + g.sum() + P.t_b * f0 + P.t_a * g0
    assert ob["cost_total"] - eps * ob["entropy"] == pytest.approx(dual, rel=1e-10, abs=1e-10)
    assert ob["mass"] == pytest.approx(P.I + P.t_b, rel=1e-12)
    # the inlier part alone: total minus the bins at their costs
    rows, row0, cols, col0 = sinkhorn.marginals(P, f, g, f0, g0, eps)
    q_i0 = np.exp((f + g0 - P.c_out) / eps)
    q_0j = np.exp((f0 + g - P.c_unm) / eps)
    q_00 = math.exp((f0 + g0 - P.c_sink) / eps)
    assert ob["cost_inlier"] == pytest.approx(
        ob["cost_total"] - P.c_out * q_i0.sum() - P.c_unm * q_0j.sum() - P.c_sink * q_00, rel=1e-12, abs=1e-12)


def test_objectives_duality_away_from_convergence_with_masked_entries():
    """Away from the fixed point the same identity holds with the actual
    marginals; entries masked out by the sparse assignment (c = +inf) carry no
    mass and no entropy."""
    rng = np.random.default_rng(5)
    P = sparse.masked_problem(_rand_problem(rng, [(6, 7), (5, 3)], c_out=1.5), 2)
    eps = 0.4
    sol = sinkhorn.solve(P, eps, tol=1e-3, n_max=3)
    f, g, f0, g0 = sol["f"], sol["g"], sol["f0"], sol["g0"]
    rows, row0, cols, col0 = sinkhorn.marginals(P, f, g, f0, g0, eps)
    ob = sinkhorn.objectives(P, f, g, f0, g0, eps)
    dual = f @ rows + g @ cols + f0 * row0 + g0 * col0
    assert ob["cost_total"] - eps * ob["entropy"] == pytest.approx(dual, rel=1e-11, abs=1e-11)
    assert ob["mass"] == pytest.approx(rows.sum() + row0, rel=1e-12)


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("t_b,eps_p", [(1.0, 0.5), (3.0, 2.0), (1.0, 8.0)])
def test_objectives_one_entry_plus_bins_closed_form(t_b, eps_p):
    """One detected spot and one model spot with the outlier row and column.
    The plan is [[x, 1 - x], [1 - x, T_b - 1 + x]] (rows: spot, row 0; columns:
    spot, column 0; T_a = T_b) and the entropic optimum fixes the cross ratio
    x (T_b - 1 + x) / (1 - x)^2 = exp((L_11 + L_00 - L_10 - L_01)/eps_p)
    (Eq. elbo).  The likelihoods are written from the paper's definitions on
    two unit rays at a known angle: L_11 = rhat.r / sigma^2, L_10 = L_00 =
    cos(3 sigma) / sigma^2 (a 3-sigma miss), L_01 = 1 / sigma^2 (the null
    angle), sigma = sigma_mm / D."""
    sigma_mm = 1.0
    sig = sigma_mm / D
    ang = 1.7 * sig
    r = _unit([-1.0, 0.2, 0.1])
    axis = _unit(np.cross(r, [0.0, 0.0, 1.0]))
    rhat = r * math.cos(ang) + np.cross(axis, r) * math.sin(ang)       # r turned by ang about axis
    L11 = float(rhat @ r) / sig ** 2
    Lout = math.cos(3.0 * sig) / sig ** 2
    Lnull = 1.0 / sig ** 2
    K = math.exp((L11 + Lout - Lout - Lnull) / eps_p)
    # (1 - K) x^2 + (T_b - 1 + 2K) x - K = 0, the root in (0, 1), cancellation-free form
    bq = t_b - 1.0 + 2.0 * K
    x = 2.0 * K / (bq + math.sqrt(bq * bq + 4.0 * K * (1.0 - K)))
    Q = np.array([[x, 1.0 - x], [1.0 - x, t_b - 1.0 + x]])
    Lmat = np.array([[L11, Lout], [Lnull, Lout]])
    H = -float(np.sum(Q * np.log(Q)))
    # the oracle: costs in mm^2 on the same rays, eps = 2 sigma_mm^2 eps_p
    c11 = D * D * float(np.sum((rhat - r) ** 2))
    eps = 2.0 * sigma_mm ** 2 * eps_p
    c_out = cost.c_out(sigma_mm, D)
    P = sinkhorn.Problem([np.array([[c11]])], c_out, 0.0, c_out, t_b)
    sol = sinkhorn.solve(P, eps, tol=1e-14, n_max=100000)
    ob = sinkhorn.objectives(P, sol["f"], sol["g"], sol["f0"], sol["g0"], eps, sigma_mm, D)
    assert ob["mass"] == pytest.approx(Q.sum(), rel=1e-12)
    assert ob["cost_inlier"] == pytest.approx(c11 * x, rel=1e-9)
    assert ob["cost_total"] == pytest.approx(c11 * x + c_out * (1.0 - x) + c_out * (t_b - 1.0 + x), rel=1e-9)
    assert ob["entropy"] == pytest.approx(H, rel=1e-9)
    assert ob["sem_objective"] == pytest.approx(float(np.sum(Lmat * Q)) + eps_p * H, rel=1e-11)


def test_gauge_shift_leaves_plan_and_dual_unchanged():
    """(f - C, g + C, f_0 - C, g_0 + C) is the same plan: every entry depends on
    a sum of one row and one column potential, and the dual value changes by
    C (|J| + T_a - |I| - T_b) = 0 with T_a = T_b + |I| - |J|.  A warm start is
    re-centred to f_0 = 0 and the solve ends at the same plan."""
    rng = np.random.default_rng(9)
    P = _rand_problem(rng, [(5, 4), (3, 6), (6, 5)], c_out=1.2)
    eps = 0.3
    s1 = sinkhorn.solve(P, eps, tol=1e-12, n_max=100000)
    C = 271.3
    f, g, f0, g0 = s1["f"] + C, s1["g"] - C, s1["f0"] + C, s1["g0"] - C
    for a, b in zip(sinkhorn.plan_blocks(P, f, g, eps), sinkhorn.plan_blocks(P, s1["f"], s1["g"], eps)):
        assert np.allclose(a, b, rtol=1e-10, atol=1e-14)
    assert sinkhorn.dual_value(P, f, g, f0, g0, eps) == pytest.approx(
        sinkhorn.dual_value(P, s1["f"], s1["g"], s1["f0"], s1["g0"], eps), rel=1e-12)
    s2 = sinkhorn.solve(P, eps, tol=1e-12, n_max=100000, f=f, g=g, f0=f0, g0=g0)
    assert s2["f0"] == pytest.approx(0.0, abs=1e-9) and s2["n_iter"] <= 2
    for a, b in zip(sinkhorn.plan_blocks(P, s2["f"], s2["g"], eps), sinkhorn.plan_blocks(P, s1["f"], s1["g"], eps)):
        assert np.allclose(a, b, rtol=1e-8, atol=1e-12)


# ---------------------------------------------------------------- pair features

def _one_rotation_geometry():
    return forward.Geometry(1, math.radians(3.0), (ig.TRANSMISSION_150, ig.BACKSCATTER_150), 1.0, 4.0)


def test_pair_features_on_a_constructed_pair():
    """Grain at R = I, x = 0, rotation 0.  Plane (2,0,0) reflects the beam
    straight back to the backscatter detector centre (sin theta = 1); plane
    (4,1,1) sends r = (-7/9, -4/9, -4/9) to (-150, -600/7, -600/7) mm
    (sin theta = 2 sqrt(2)/3).  The spot normals are (1,0,0) and (4,1,1)/sqrt 18
    (cos = 4/sqrt 18).  Every feature of every hypothesis of this pair is
    written here from the plane indices and this geometry."""
    pl = crystal.cubic_planes(A_BCC, "I", 30)
    g = _one_rotation_geometry()
    p12 = np.array([[0.0, 0.0], [-600.0 / 7.0, -600.0 / 7.0]])
    off = np.array([0, 0, 2])                        # block 0 transmission (empty), 1 backscatter
    c = candidates.generate(pl, g, p12, off, 1, 0, delta_deg=1.5, pairs=(np.array([0]), np.array([1])))
    assert len(c["ma"]) > 0
    delta = math.radians(1.5)
    cos_n = 4.0 / math.sqrt(18.0)
    ang_n = math.acos(cos_n)
    sth_a, sth_b = 1.0, 2.0 * math.sqrt(2.0) / 3.0
    sep = 600.0 * math.sqrt(2.0) / 7.0
    hkl = pl["hkl"].astype(np.float64)
    nsq = np.sum(hkl ** 2, axis=1)
    for k in range(len(c["ma"])):
        ma, mb = int(c["ma"][k]), int(c["mb"][k])
        wa, wb = hkl[ma] / math.sqrt(nsq[ma]), hkl[mb] / math.sqrt(nsq[mb])
        lam_a = 2.0 * A_BCC / math.sqrt(nsq[ma]) * sth_a
        lam_b = 2.0 * A_BCC / math.sqrt(nsq[mb]) * sth_b
        expect = [cos_n, wa @ wb, abs(math.acos(np.clip(wa @ wb, -1, 1)) - ang_n) / delta, sth_a, sth_b,
                  (lam_a - 1.0) / 3.0, (lam_b - 1.0) / 3.0, nsq[ma] / 30.0, nsq[mb] / 30.0,
                  sep / 400.0, 0.0, sep / 200.0, 1.0, 1.0]
        assert np.allclose(c["feat"][k], expect, rtol=0, atol=1e-12), (ma, mb)
        assert 1.0 <= lam_a <= 4.0 and 1.0 <= lam_b <= 4.0
        assert abs(math.acos(np.clip(wa @ wb, -1, 1)) - ang_n) <= delta
    # the hypothesis ({200}, {411}) recovers the grain (up to cubic symmetry)
    mis = np.degrees(metrics.misorientation(c["q"], np.array([1.0, 0.0, 0.0, 0.0])))
    assert mis.min() < 1e-9


# ---------------------------------------------------------------- SPOT values

def test_single_score_lbar_closed_form_and_unmatched():
    """A candidate at R = I, x = 0 with three model spots on the backscatter
    detector at rotation 0: (2,0,0) at the centre, (4,1,1) at (-600/7,
    -600/7) and (5,1,0) at (-62.5, 0) mm.  Detected spots sit at known offsets
    from the first two; none is near (5,1,0).  Each entry of the SPOT column
    is ln sum_j exp(-c_ij / (2 sigma^2)) with c_ij = D^2 |rhat_i - r_j|^2 from
    the unit rays, kept when above the floor -c_out / (2 sigma^2); exactly one
    model spot is unmatched."""
    pl = crystal.cubic_planes(A_BCC, "I", 30)
    g = _one_rotation_geometry()
    idx = {tuple(h): i for i, h in enumerate(pl["hkl"].tolist())}
    ms = [idx[(2, 0, 0)], idx[(4, 1, 1)], idx[(5, 1, 0)]]
    model = {"m": np.array(ms), "n": np.zeros(3, np.int64), "t": np.zeros(3, np.int64),
             "det": np.ones(3, np.int64), "block": np.ones(3, np.int64), "offsets": np.array([0, 0, 3])}
    rays = np.array([[-1.0, 0.0, 0.0], [-7.0 / 9, -4.0 / 9, -4.0 / 9], [-150.0, -62.5, 0.0]])
    rays = rays / np.linalg.norm(rays, axis=1, keepdims=True)
    sb = np.array([[0.0, 0.0], [-600.0 / 7.0, -600.0 / 7.0]])
    offs = [(0.0, 0.0), (0.4, -0.3), (1.5, 1.0), (4.0, 0.0), (-2.0, 2.5)]
    p12 = np.array([sb[k] + np.array(o) for k in (0, 1) for o in offs])
    sigma = 1.0
    c_out = cost.c_out(sigma, D)
    q = np.array([1.0, 0.0, 0.0, 0.0])
    un, nm, rows, vals = single.score(pl, g, D, p12, np.array([0, 0, len(p12)]), model, q, np.zeros(3),
                                      sigma, c_out)
    assert nm == 3 and un == 1
    lab = np.c_[np.full(len(p12), -150.0), p12]
    rhat = lab / np.linalg.norm(lab, axis=1, keepdims=True)
    cmat = D * D * np.sum((rhat[:, None, :] - rays[None, :, :]) ** 2, axis=-1)
    lbar = np.logaddexp.reduce(-cmat / (2.0 * sigma ** 2), axis=1)
    keep = np.nonzero(lbar > -c_out / (2.0 * sigma ** 2))[0]
    assert 0 < len(keep) < len(p12)
    assert np.array_equal(rows, keep)
    assert np.allclose(vals, lbar[keep], rtol=1e-10, atol=1e-10)
    # on the model spot itself the value is 0 (one term, zero cost)
    assert vals[0] == pytest.approx(0.0, abs=1e-9)


# ---------------------------------------------------------------- annealing modes

def test_cooling_schedules():
    s = em.cooling_schedule(100.0, 2.0, 0.97)
    assert s[0] == 100.0 and s[-1] <= 2.0 < s[-2]
    assert np.allclose(np.array(s[1:]) / np.array(s[:-1]), 0.97, rtol=1e-15)
    assert len(s) == math.ceil(math.log(100.0 / 2.0) / -math.log(0.97)) + 1
    r = single.cooling_schedule(30.0, 5, 0.97)
    assert r == pytest.approx([30.0 * 0.97 ** k for k in range(5)], rel=1e-15)
    with pytest.raises(ValueError):
        em.cooling_schedule(1.0, 2.0, 1.5)


def _noise_free_problem(n_grains=2, n_rot=6, seed=11):
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry(n_rot, np.deg2rad(30.0), p.detectors, p.lam_min, p.lam_max)
    q, x = ig.random_grains(p, n=n_grains, seed=seed)
    sim = simulate.simulate(pl, q, x, g, 0.0, 0.0, seed, p.distance)
    return p, pl, g, q, x, sim


def test_paper_annealing_em_stops_on_plan_change():
    """Alg. LaueOT with the cooling rule: eps x cool per EM iteration down to the
    floor 2 sigma^2 (eps_p = 1; a coarse cool keeps the test short), then EM
    iterations at that temperature until ||Q^{k+1} - Q^k||_F <= zeta_tol.  The
    run equals a plain run over the same temperatures cut after the first
    iteration under the tolerance, the plan change falls geometrically at the
    last temperature, and the grains end near the truth (0.3 mm noise)."""
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry(6, np.deg2rad(30.0), p.detectors, p.lam_min, p.lam_max)
    q, x = ig.random_grains(p, n=2, seed=11)
    sim = simulate.simulate(pl, q, x, g, 0.3, 0.1, 11, p.distance)
    q0, x0 = ig.perturb_grains(q, x, 1.0, 1.0, 5)
    model = forward.enumerate_visible(pl, q0, x0, g)
    model["offsets"] = forward.block_offsets(model["block"], g.n_blocks)
    sig2 = 0.3 ** 2
    c_out = cost.c_out(0.3, p.distance)
    sched = em.cooling_schedule(20.0 * sig2, 2.0 * sig2, 0.7)
    res = em.run(pl, g, p.distance, sim["p12"], sim["offsets"], model, q0, x0, sched, c_out,
                 tol=1e-12, n_max=20000, zeta_tol=1e-6, n_final_max=40)
    st = res["stats"]
    n = len(st)
    assert len(sched) + 3 < n < len(sched) + 40
    assert st[-1]["zeta"] <= 1e-6 and all(s["zeta"] > 1e-6 for s in st[len(sched) - 1:-1])
    assert [s["eps"] for s in st] == sched + [sched[-1]] * (n - len(sched))
    z = np.array([s["zeta"] for s in st[len(sched):]])
    assert np.all(z[1:] < z[:-1])
    plain = em.run(pl, g, p.distance, sim["p12"], sim["offsets"], model, q0, x0, [s["eps"] for s in st], c_out,
                   tol=1e-12, n_max=20000)
    assert np.array_equal(plain["q"], res["q"]) and np.array_equal(plain["x"], res["x"])
    assert np.max(np.degrees(metrics.misorientation(res["q"], q))) < 0.2      # the noise is 0.11 deg per ray
    assert np.max(np.linalg.norm(res["x"] - x, axis=1)) < 0.6      # six rotations fix positions loosely


def test_paper_single_refinement_schedule_recovers_noise_free_grain():
    """Alg. SingleLaueOT with eps_init x 0.97^k for k_max iterations and four
    Gauss-Newton steps per iteration (App. D) pulls a start 1 deg / 0.3 mm off
    onto the noise-free grain."""
    p, pl, g, q, x, sim = _noise_free_problem(n_grains=1, seed=4)
    q0, x0 = ig.perturb_grains(q, x, 1.0, 0.3, 8)
    eps_list = single.cooling_schedule(30.0 * 0.09, 60, 0.94)
    qq, xx, _ = single.refine(pl, g, p.distance, sim["p12"], sim["offsets"], q0[0], x0[0], 0.3,
                              cost.c_out(0.3, p.distance), k_gn=4, eps_list=eps_list)
    assert np.degrees(metrics.misorientation(qq, q[0])) < 1e-6
    assert np.linalg.norm(xx - x[0]) < 1e-6
