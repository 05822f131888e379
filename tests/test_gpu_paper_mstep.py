"""The paper's coordinate-descent M-step on the GPU (LauePosNewton on x, then
LaueRotMM on R; App. B) against the oracle's (oracle/mstep.py paper_step)
on identical FP32 inputs: one M-step from the same plan, the EM, the sparse
EM, batching, and the argument checks."""
import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import cost, metrics, mstep, sinkhorn
from oracle import em as oem
from tests import _problems

pytestmark = pytest.mark.gpu

CASES = [("tiny", None, None, 0), ("medium", 4, 60, 0), ("medium", 3, 100, 1)]
KW = {"k_newton": 3, "tol_x": 1e-9, "k_mm": 500, "tol_r": 1e-12}
ORACLE_KW = {"n_newton": 3, "tol_x": 1e-9, "n_mm": 500, "tol_r": 1e-12}


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-T{c[1]}-N{c[2]}")
def prob(request):
    name, n_rot, n_grains, shift = request.param
    return _problems.make(ig.PRESETS[name], n_rot=n_rot, n_grains=n_grains, seed_shift=shift)


def _plan_pairs(prob, eps):
    p = prob.preset
    t_b = sinkhorn.default_tb(len(prob.model["m"]))
    c_out = cost.c_out(p.sigma_mm, p.distance)
    C = _problems.oracle_costs(prob)
    P = sinkhorn.Problem(C, c_out, 0.0, c_out, t_b)
    ref = sinkhorn.solve(P, eps, tol=1e-6, n_max=5000)
    f32, g32 = ig.to_f32_exact(ref["f"]), ig.to_f32_exact(ref["g"])
    Qb = sinkhorn.plan_blocks(P, f32, g32, eps)
    p_lab = oem.obs_lab(prob.geom, prob.obs["p12"], prob.obs["block"])
    pairs = oem.grain_pairs(prob.planes, prob.geom, p_lab, prob.obs["offsets"], prob.model, Qb, len(prob.q0))
    return pairs, f32, g32, c_out, t_b


def test_paper_mstep_matches_oracle(gpu_lib, prob):
    laue = gpu_lib
    p = prob.preset
    eps = 11.1 * p.sigma_mm ** 2
    pairs, f32, g32, c_out, t_b = _plan_pairs(prob, eps)
    q_or, x_or = prob.q0.copy(), prob.x0.copy()
    q_gn, x_gn = prob.q0.copy(), prob.x0.copy()
    for n, pr in enumerate(pairs):
        if pr is not None:
            q_or[n], x_or[n] = mstep.paper_step(pr, q_or[n], x_or[n], prob.geom, **ORACLE_KW)
            q_gn[n], x_gn[n], *_ = mstep.gn_step(pr, q_gn[n], x_gn[n], prob.geom, p.distance)
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    grains = laue.Grains(prob.q0, prob.x0)
    f = torch.tensor(f32, dtype=torch.float32, device="cuda")
    g = torch.tensor(g32, dtype=torch.float32, device="cuda")
    ot = laue.ot_params(eps, p.distance, c_out, t_b)
    steps = laue.laue_mstep(geom, planes, obs, model, ot, f, g, grains, k_gn=1, mstep="paper", **KW)
    qg, xg = grains.numpy()
    mis = np.degrees(metrics.misorientation(qg, q_or))
    dx = np.linalg.norm(xg - x_or, axis=1)
    assert np.max(mis) < 2e-4, np.max(mis)
    assert np.max(dx) < 2e-4, np.max(dx)
    assert torch.all(torch.isfinite(steps))
    # the two oracle routes differ by far more than the GPU's distance to the paper's
    sep = np.degrees(metrics.misorientation(q_gn, q_or)) + np.linalg.norm(x_gn - x_or, axis=1)
    big = sep > 50 * 2e-4
    assert big.any()
    assert np.all((mis + dx)[big] < 0.1 * sep[big])


def _em_both(laue, P, rho=0, k_gn=1):
    p = P.preset
    c_out = cost.c_out(p.sigma_mm, p.distance)
    t_b = sinkhorn.default_tb(len(P.model["m"]))
    eps_list = oem.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    ref = oem.run(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model, P.q0, P.x0, eps_list,
                  c_out, t_b=t_b, k_gn=k_gn, tol=1e-5, n_max=2000, rho=rho or None, mstep_method="paper",
                  paper_kw=ORACLE_KW)
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    ot = laue.ot_params(p.eps_start, p.distance, c_out, t_b, tol=1e-5, n_max=2000, rho=rho)
    par = laue.em_params(ot, p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage, k_gn=k_gn, mstep="paper", **KW)
    gr = laue.Grains(P.q0, P.x0)
    out = laue.laue_em(geom, planes, obs, model, par, gr)
    return ref, out, gr


@pytest.mark.parametrize("rho", [0, 8])
def test_paper_em_matches_oracle(gpu_lib, rho):
    laue = gpu_lib
    P = _problems.make(ig.TINY)
    ref, out, gr = _em_both(laue, P, rho)
    qg, xg = gr.numpy()
    assert out["code"] == 0 and out["n_em_iter"] == 20 and out["not_converged"] == 0
    assert np.max(np.degrees(metrics.misorientation(qg, ref["q"]))) < 0.01
    assert np.max(np.linalg.norm(xg - ref["x"], axis=1)) < 0.01
    assert np.max(np.degrees(metrics.misorientation(qg, P.q_true))) < 0.1
    # one sweep streams k_newton position passes and one rotation pass per EM iteration
    assert out["mstep_entries"] > 0


def test_paper_em_noise_free_recovery(gpu_lib):
    laue = gpu_lib
    P = _problems.make(ig.TINY, sigma=0.0, frac=0.0, seed_shift=3)
    ref, out, gr = _em_both(laue, P, k_gn=4)
    qg, xg = gr.numpy()
    assert np.max(np.degrees(metrics.misorientation(qg, P.q_true))) < 2e-3
    assert np.max(np.linalg.norm(xg - P.x_true, axis=1)) < 2e-3


def test_paper_batched_equals_solo(gpu_lib):
    laue = gpu_lib
    from tests.test_gpu_batch import _sample
    presets = ig.batching_samples(3)
    samples = [_sample(laue, pr, int(g), k) for k, (pr, g) in enumerate(zip(presets, (11, 24, 5)))]
    for k, s in enumerate(samples):
        s[5].gn = laue.gn_params(1, 1e-9, mstep="paper", k_newton=3, k_mm=200 + 100 * k, tol_x=1e-9, tol_r=1e-12)
    seq = []
    for p, geom, planes, obs, model, par, (q0, x0), _ in samples:
        gr = laue.Grains(q0, x0)
        out = laue.laue_em(geom, planes, obs, model, par, gr)
        seq.append((gr.numpy(), out))
    grains = [laue.Grains(*s[6]) for s in samples]
    rc, outs = laue.laue_em_batched([s[1] for s in samples], [s[2] for s in samples], [s[3] for s in samples],
                                    [s[4] for s in samples], [s[5] for s in samples], grains)
    for k in range(len(samples)):
        (qs, xs), o1 = seq[k]
        qb, xb = grains[k].numpy()
        assert np.array_equal(qs, qb) and np.array_equal(xs, xb), k
        for key in ("f", "g", "j_star"):
            assert torch.equal(o1[key][:outs[k][key].numel()], outs[k][key]), (k, key)


def test_paper_mstep_argument_checks(gpu_lib):
    laue = gpu_lib
    P = _problems.make(ig.TINY)
    p = P.preset
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    f = torch.zeros(obs.n, dtype=torch.float32, device="cuda")
    g = torch.zeros(model.n, dtype=torch.float32, device="cuda")
    ot = laue.ot_params(11.1 * p.sigma_mm ** 2, p.distance, cost.c_out(p.sigma_mm, p.distance), 10.0)
    for kw in ({"k_newton": 0}, {"k_mm": 0}, {"tol_x": -1.0}, {"tol_r": float("nan")}):
        with pytest.raises(laue.LaueError) as e:
            laue.laue_mstep(geom, planes, obs, model, ot, f, g, laue.Grains(P.q0, P.x0), k_gn=1, mstep="paper",
                            **kw)
        assert e.value.code == -1, kw
    gn = laue.gn_params(1, mstep="paper")
    gn.method = 2
    par = laue.em_params(ot, 1.0, 1.0, 1, 1)
    par.gn = gn
    with pytest.raises(laue.LaueError) as e:
        laue.laue_em(geom, planes, obs, model, par, laue.Grains(P.q0, P.x0))
    assert e.value.code == -1
    # more planes than the rotation step holds
    many = laue.laue_planes_cubic(p.a, p.centering, 200)
    assert many.n > 1024
    with pytest.raises(laue.LaueError) as e:
        laue.laue_mstep(geom, many, obs, model, ot, f, g, laue.Grains(P.q0, P.x0), k_gn=1, mstep="paper")
    assert e.value.code == -1
    # with k_gn = 0 nothing moves
    gr = laue.Grains(P.q0, P.x0)
    laue.laue_mstep(geom, planes, obs, model, ot, f, g, gr, k_gn=0, mstep="paper")
    q1, x1 = gr.numpy()
    assert np.array_equal(q1, P.q0) and np.array_equal(x1, P.x0)
