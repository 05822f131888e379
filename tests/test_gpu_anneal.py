"""GPU parity of the paper's annealing modes and of the EM's outputs at its
last E-step: Alg. LaueOT's cooling with the plan-change stop, Alg.
SingleLaueOT's cooling in the single-grain refinement, the sparse
assignment's first temperature, and the assignments, Q_0j and likelihood of
the last plan, all against the oracle."""
import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import candidates, cost, em as oem, metrics, single, sinkhorn, sparse
from tests import _problems

pytestmark = pytest.mark.gpu


def _gpu_em(laue, P, par, grains=None):
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    grains = laue.Grains(P.q0, P.x0) if grains is None else grains
    out = laue.laue_em(geom, planes, obs, model, par, grains)
    return out, grains


def _gpu_costs(laue, P, grains):
    """Oracle cost blocks on the library's FP32 model-spot geometry at grains
    (laue_forward_eval), so that plan comparisons are stage-isolated."""
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    laue.laue_forward_eval(geom, planes, grains, model)
    m = model.numpy()
    s12 = np.stack([m["s1"], m["s2"]], axis=1).astype(np.float64)
    vloc = np.stack([m["vn"], m["v1"], m["v2"]], axis=1).astype(np.float64)
    off, mo = P.obs["offsets"], P.model["offsets"]
    return [cost.chord_cost(P.obs["p12"][off[b]:off[b + 1]], s12[mo[b]:mo[b + 1]], vloc[mo[b]:mo[b + 1]],
                            P.preset.distance) for b in range(P.geom.n_blocks)]


def _cooling_case():
    P = _problems.make(ig.TINY, n_rot=8, seed_shift=21, perturb=(1.0, 1.0))
    p = P.preset
    s2 = p.sigma_mm ** 2
    return P, p, 20.0 * s2, 2.0 * s2, 0.7


def _plan_change_stop_case(laue, P, p, e0, e1, cool, rho, k):
    """Temperatures eps_start cool^i down to e1, then EM iterations at the
    last one until ||Q^{k+1} - Q^k||_F <= zeta_tol.  zeta_tol is placed
    halfway (geometrically) between two of the oracle's plan changes, so both
    sides stop at the same iteration; grains within 0.01 deg, 2e-3 mm, the
    last plan change within 1e-3 relative.  rho > 0: the sparse assignment
    on both sides (the plans are 0 off each detected spot's rho nearest model
    spots, re-chosen at every E-step)."""
    c_out = cost.c_out(p.sigma_mm, p.distance)
    t_b = sinkhorn.default_tb(len(P.model["m"]))
    sched = oem.cooling_schedule(e0, e1, cool)
    kw = {"rho": rho} if rho else {}
    probe = oem.run(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model, P.q0, P.x0, sched,
                    c_out, t_b=t_b, tol=1e-5, n_max=2000, zeta_tol=0.0, n_final_max=12, **kw)
    z = [s["zeta"] for s in probe["stats"][len(sched):]]
    assert z[k] < z[k - 1] / 1.5
    zeta_tol = float(np.sqrt(z[k] * z[k - 1]))
    ref = oem.run(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model, P.q0, P.x0, sched, c_out,
                  t_b=t_b, tol=1e-5, n_max=2000, zeta_tol=zeta_tol, n_final_max=12, **kw)
    ot = laue.ot_params(e0, p.distance, c_out, t_b, tol=1e-5, n_max=2000, rho=rho)
    par = laue.em_params(ot, e0, e1, 1, 1, eps_cool=cool, final_iters=12, zeta_tol=zeta_tol, sigma_mm=p.sigma_mm)
    out, grains = _gpu_em(laue, P, par)
    assert out["n_em_iter"] == len(ref["stats"]) == len(sched) + k + 1
    assert out["final_iters_run"] == k + 1
    # the two EMs' plans agree entry by entry within 1e-4, so their plan
    # changes within 1e-4 sqrt(2 |I|) (Frobenius norm of the difference)
    assert abs(out["zeta"] - ref["stats"][-1]["zeta"]) <= 1e-4 * np.sqrt(2.0 * len(P.obs["p12"]))
    qg, xg = grains.numpy()
    assert np.max(np.degrees(metrics.misorientation(qg, ref["q"]))) < 0.01
    assert np.max(np.linalg.norm(xg - ref["x"], axis=1)) < 2e-3
    assert out["not_converged"] == 0


def test_em_cooling_with_plan_change_stop_matches_oracle(gpu_lib):
    P, p, e0, e1, cool = _cooling_case()
    _plan_change_stop_case(gpu_lib, P, p, e0, e1, cool, 0, 4)


def test_em_cooling_with_plan_change_stop_sparse_matches_oracle(gpu_lib):
    """The same with the sparse assignment (rho = 8) on blocks of up to 40
    model spots: the plan change over the union of the two E-steps'
    neighbour sets."""
    P = _problems.make(ig.TINY, n_rot=4, n_grains=12, seed_shift=21, perturb=(1.0, 1.0))
    assert np.max(np.diff(P.model["offsets"])) > 8
    s2 = P.preset.sigma_mm ** 2
    _plan_change_stop_case(gpu_lib, P, P.preset, 20.0 * s2, 2.0 * s2, 0.7, 8, 4)


def test_plan_change_on_the_gpus_plans(gpu_lib):
    """zeta of the library against the oracle's ||Q^1 - Q^0||_F evaluated on the
    library's own two plans (stage-isolated): plan 0 = the potentials of one
    EM iteration at the start grains, plan 1 = those of the next iteration at
    the grains after its M-step (obtained by one-iteration calls, which run the
    same arithmetic as the two-iteration call)."""
    laue = gpu_lib
    P, p, e0, e1, cool = _cooling_case()
    c_out = cost.c_out(p.sigma_mm, p.distance)
    t_b = sinkhorn.default_tb(len(P.model["m"]))
    eps = 4.0 * p.sigma_mm ** 2
    ot = laue.ot_params(eps, p.distance, c_out, t_b, tol=1e-6)
    two, _ = _gpu_em(laue, P, laue.em_params(ot, eps, eps, 1, 1, eps_cool=0.5, final_iters=1))
    assert two["n_em_iter"] == 2 and two["final_iters_run"] == 1
    one, g1 = _gpu_em(laue, P, laue.em_params(ot, eps, eps, 1, 1))
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    nxt = laue.laue_em(geom, planes, obs, model, laue.em_params(ot, eps, eps, 1, 1), g1, one["f"].clone(),
                       one["g"].clone(), one["f0"], one["g0"])
    assert torch.equal(nxt["f"], two["f"]) and torch.equal(nxt["g"], two["g"])
    # grains after the first M-step: repeat the one-iteration call
    _, gb = _gpu_em(laue, P, laue.em_params(ot, eps, eps, 1, 1))
    plans = []
    for res, grains in ((one, laue.Grains(P.q0, P.x0)), (nxt, gb)):
        Pr = sinkhorn.Problem(_gpu_costs(laue, P, grains), c_out, 0.0, c_out, t_b)
        f, g = res["f"].double().cpu().numpy(), res["g"].double().cpu().numpy()
        Qb = sinkhorn.plan_blocks(Pr, f, g, eps)
        bins = (np.exp((f + res["g0"] - c_out) / eps), np.exp((res["f0"] + g) / eps),
                np.array([np.exp((res["f0"] + res["g0"] - c_out) / eps)]))
        plans.append((Qb, bins))
    z = oem.plan_change(plans[1][0], plans[1][1], plans[0][0], plans[0][1])
    assert z > 1e-3
    assert two["zeta"] == pytest.approx(z, rel=1e-3)


def test_em_cooling_runs_every_final_iteration_without_tolerance(gpu_lib):
    laue = gpu_lib
    P, p, e0, e1, cool = _cooling_case()
    c_out = cost.c_out(p.sigma_mm, p.distance)
    t_b = sinkhorn.default_tb(len(P.model["m"]))
    n_temps = len(oem.cooling_schedule(e0, e1, cool))
    ot = laue.ot_params(e0, p.distance, c_out, t_b)
    out, _ = _gpu_em(laue, P, laue.em_params(ot, e0, e1, 1, 1, eps_cool=cool, final_iters=3))
    assert out["n_em_iter"] == n_temps + 3 and out["final_iters_run"] == 3
    # the sparse assignment too (the plan change is recorded, nothing stops)
    ot32 = laue.ot_params(e0, p.distance, c_out, t_b, rho=8)
    out, _ = _gpu_em(laue, P, laue.em_params(ot32, e0, e1, 1, 1, eps_cool=cool, final_iters=2))
    assert out["n_em_iter"] == n_temps + 2 and np.isfinite(out["zeta"])


def test_em_outputs_are_those_of_the_last_estep(gpu_lib):
    """One EM iteration (E-step, then the M-step moves the grains): the hard
    assignments, Q_0j and the likelihood come from the E-step's plan, i.e. the
    GPU's potentials at the starting geometry, evaluated here by the oracle
    (stage-isolated: the oracle consumes the GPU's FP32 potentials)."""
    laue = gpu_lib
    P = _problems.make(ig.TINY, seed_shift=5)
    p = P.preset
    c_out = cost.c_out(p.sigma_mm, p.distance)
    t_b = sinkhorn.default_tb(len(P.model["m"]))
    eps = 0.6
    ot = laue.ot_params(eps, p.distance, c_out, t_b, tol=1e-6)
    out, grains = _gpu_em(laue, P, laue.em_params(ot, eps, eps, 1, 1, k_gn=2, sigma_mm=p.sigma_mm))
    qg, _ = grains.numpy()
    assert np.max(np.degrees(metrics.misorientation(qg, P.q0))) > 1e-3       # the M-step moved the grains
    Pr = sinkhorn.Problem(_gpu_costs(laue, P, laue.Grains(P.q0, P.x0)), c_out, 0.0, c_out, t_b)
    f = out["f"].double().cpu().numpy()
    g = out["g"].double().cpu().numpy()
    js, qs, qi0 = sinkhorn.hard_assignment(Pr, f, g, out["f0"], out["g0"], eps)
    # decisions agree wherever the two best entries are not within 1e-4 of each other
    Qb = sinkhorn.plan_blocks(Pr, f, g, eps)
    margin = np.empty(Pr.I)
    for b, q in enumerate(Qb):
        r0, r1 = Pr.row_off[b], Pr.row_off[b + 1]
        allq = np.concatenate([q, qi0[r0:r1, None]], axis=1) if q.shape[1] else qi0[r0:r1, None]
        srt = -np.sort(-allq, axis=1)
        margin[r0:r1] = srt[:, 0] - (srt[:, 1] if allq.shape[1] > 1 else 0.0)
    clear = margin > 1e-4
    assert clear.mean() > 0.95
    assert np.array_equal(out["j_star"].cpu().numpy()[clear], js[clear])
    assert np.allclose(out["q_star"].cpu().numpy(), qs, rtol=1e-4, atol=1e-6)
    assert np.allclose(out["q_out"].cpu().numpy(), qi0, rtol=1e-4, atol=1e-6)
    q0j = np.exp((out["f0"] + g - 0.0) / eps)
    assert np.allclose(out["q_unm"].cpu().numpy(), q0j, rtol=1e-5, atol=1e-7)
    ob = sinkhorn.objectives(Pr, f, g, out["f0"], out["g0"], eps, p.sigma_mm, p.distance)
    o = out["objective"]
    assert o["mass"] == pytest.approx(ob["mass"], rel=2e-5)
    assert o["cost_total"] == pytest.approx(ob["cost_total"], rel=2e-5)
    assert o["entropy"] == pytest.approx(ob["entropy"], rel=1e-4)
    assert o["sem_objective"] == pytest.approx(ob["sem_objective"], rel=1e-5)
    # without sigma_mm no likelihood is computed
    out2, _ = _gpu_em(laue, P, laue.em_params(ot, eps, eps, 1, 1, k_gn=2))
    assert np.isnan(out2["objective"]["sem_objective"])


def test_refinement_cooling_matches_oracle(gpu_lib):
    """Alg. SingleLaueOT's temperatures eps_init cool^k for k_max iterations with
    four Gauss-Newton steps each (App. D), on candidates near true grains and
    random ones: refined grains within 1e-3 deg and 2e-3 mm of the oracle's."""
    laue = gpu_lib
    p = ig.MEDIUM
    from tests.test_gpu_index import _setup
    _, pl, g, q, x, sim, p12, geom, planes, obs = _setup(laue)
    ref = candidates.generate(pl, g, p12, sim["offsets"], 200, 5)
    mis = np.degrees(metrics.misorientation(ref["q"][:, None, :], q[None, :, :])).min(axis=1)
    sel = np.concatenate([np.argsort(mis)[:4], np.arange(0, len(mis), max(1, len(mis) // 4))[:4]])
    cq, cx = ref["q"][sel], np.zeros((len(sel), 3))
    c_out = cost.c_out(p.sigma_mm, p.distance)
    e0, k_max, cool = 60.0 * p.sigma_mm ** 2, 24, 0.85
    eps_list = single.cooling_schedule(e0, k_max, cool)
    grains = laue.Grains(cq, cx)
    par = laue.score_params(p.sigma_mm, p.distance, c_out, k_refine=k_max, k_gn=4, chunk=8, eps_start=e0,
                            eps_cool=cool)
    laue.laue_score_candidates(geom, planes, obs, grains, par)
    qg, xg = grains.numpy()
    for k in range(len(sel)):
        qq, xx, _ = single.refine(pl, g, p.distance, p12, sim["offsets"], cq[k], cx[k], p.sigma_mm, c_out,
                                  k_gn=4, eps_list=eps_list)
        assert np.degrees(metrics.misorientation(qg[k], qq)) < 1e-3
        assert np.linalg.norm(xg[k] - xx) < 2e-3


@pytest.mark.parametrize("rho", [8, 32])
def test_eps_init_matches_oracle(gpu_lib, rho):
    """The sparse assignment's first temperature: median farthest-neighbour
    chord cost over ln 100 (Sec. 7), against the oracle's on the same FP32
    column data."""
    laue = gpu_lib
    P = _problems.make(ig.MEDIUM, n_rot=6, n_grains=40, seed_shift=2)
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    ot = laue.ot_params(1.0, P.preset.distance, cost.c_out(1.0, P.preset.distance), 0.0, rho=rho)
    e = laue.laue_eps_init(geom, obs, model, ot)
    ref = sparse.eps_init(_problems.oracle_costs(P), rho)
    assert e == pytest.approx(ref, rel=1e-5)
