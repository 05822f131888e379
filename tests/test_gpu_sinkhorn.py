"""GPU parity of the cost, the streamed Sinkhorn and the M-step, stage by
stage, against the oracle on identical FP32 inputs."""
import math

import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import cost, crystal, metrics, mstep, sinkhorn
from oracle import em as oem
from tests import _problems

pytestmark = pytest.mark.gpu

CASES = [("tiny", None, None, 0), ("medium", 4, 60, 0), ("medium", 3, 100, 1)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-T{c[1]}-N{c[2]}")
def prob(request):
    name, n_rot, n_grains, shift = request.param
    return _problems.make(ig.PRESETS[name], n_rot=n_rot, n_grains=n_grains, seed_shift=shift)


def test_cost_matches_oracle(gpu_lib, prob):
    laue = gpu_lib
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    C = _problems.oracle_costs(prob)
    D = prob.preset.distance
    worst = 0.0
    for b, Cb in enumerate(C):
        if Cb.size == 0:
            continue
        G = laue.laue_cost_block(geom, obs, model, D, b).cpu().numpy().astype(np.float64)
        # accuracy contract: |c_gpu - c| <= 1e-6 c + 1e-7 mm^2 where the cost is small
        # enough to matter; relative 2e-6 everywhere
        near = Cb < 100.0
        err = np.abs(G - Cb)
        assert np.all(err[near] <= 1e-6 * Cb[near] + 1e-7 + 4e-7 * Cb[near])
        assert np.all(err <= 2e-6 * Cb + 1e-7)
        worst = max(worst, float(np.max(err / (Cb + 1e-3))))
    assert worst < 2e-6


@pytest.mark.parametrize("eps_scale", [111.0, 11.1])
def test_sinkhorn_plan_matches_oracle(gpu_lib, prob, eps_scale):
    laue = gpu_lib
    p = prob.preset
    eps = eps_scale * p.sigma_mm ** 2
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    J = model.n
    t_b = sinkhorn.default_tb(J)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    C = _problems.oracle_costs(prob)
    P = sinkhorn.Problem(C, c_out, 0.0, c_out, t_b)
    ref = sinkhorn.solve(P, eps, tol=1e-5, n_max=3000)
    ot = laue.ot_params(eps, p.distance, c_out, t_b, tol=1e-5, n_max=3000)
    f = torch.zeros(max(obs.n, 1), dtype=torch.float32, device="cuda")
    g = torch.zeros(max(model.n, 1), dtype=torch.float32, device="cuda")
    f0, g0, st, rc = laue.laue_sinkhorn(geom, obs, model, ot, f, g)
    assert st["converged"] and st["err"] <= 1e-5, st
    assert abs(st["n_iter"] - ref["n_iter"]) <= 2, (st, ref["n_iter"])
    assert f0 == pytest.approx(ref["f0"], abs=1e-3 * eps)
    assert g0 == pytest.approx(ref["g0"], abs=1e-3 * eps)
    Qref = sinkhorn.plan_blocks(P, ref["f"], ref["g"], eps)
    worst = 0.0
    for b in range(prob.geom.n_blocks):
        if Qref[b].size == 0:
            continue
        Qg = laue.laue_plan_block(geom, obs, model, ot, f, g, b).cpu().numpy()
        worst = max(worst, float(np.max(np.abs(Qg - Qref[b]))))
    assert worst <= 1e-4, worst
    # the marginal contract (row error <= 1e-5) in FP64 on the GPU's own FP32
    # costs and potentials; columns are exact after the column half up to rounding
    fg = f[:obs.n].cpu().numpy().astype(np.float64)
    gg = g[:model.n].cpu().numpy().astype(np.float64)
    Cg = [laue.laue_cost_block(geom, obs, model, p.distance, b).cpu().numpy().astype(np.float64)
          if C[b].size else C[b] for b in range(prob.geom.n_blocks)]
    Pg = sinkhorn.Problem(Cg, c_out, 0.0, c_out, t_b)
    rows, row0, cols, col0 = sinkhorn.marginals(Pg, fg, gg, f0, g0, eps)
    print(f"eps {eps:.3g}: GPU-cost marginal errors rows {np.max(np.abs(rows - 1)):.2e} "
          f"cols {np.max(np.abs(cols - 1)):.2e} row0 {abs(row0 - t_b) / t_b:.2e}")
    assert np.max(np.abs(rows - 1.0)) <= 1.05e-5
    assert abs(row0 - t_b) / t_b <= 1.05e-5
    assert np.max(np.abs(cols - 1.0)) <= 2e-6
    # on the oracle's FP64 costs of the same inputs the cost rounding (relative
    # 2e-6, i.e. 2e-6 c / eps in each exponent) adds to the error
    rows, row0, cols, col0 = sinkhorn.marginals(P, fg, gg, f0, g0, eps)
    print(f"eps {eps:.3g}: oracle-cost marginal errors rows {np.max(np.abs(rows - 1)):.2e} "
          f"cols {np.max(np.abs(cols - 1)):.2e}")
    assert np.max(np.abs(cols - 1.0)) < 3e-5
    assert np.max(np.abs(rows - 1.0)) < 3e-5


def test_sinkhorn_warm_start_and_cap(gpu_lib, prob):
    laue = gpu_lib
    p = prob.preset
    eps = 11.1 * p.sigma_mm ** 2
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    t_b = sinkhorn.default_tb(model.n)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    C = _problems.oracle_costs(prob)
    P = sinkhorn.Problem(C, c_out, 0.0, c_out, t_b)
    # warm start from a coarse solution at a larger temperature, both sides
    warm = sinkhorn.solve(P, 10 * eps, tol=1e-3, n_max=50)
    ref = sinkhorn.solve(P, eps, tol=1e-5, n_max=3000, f=warm["f"], g=warm["g"], f0=warm["f0"], g0=warm["g0"])
    f = torch.tensor(warm["f"], dtype=torch.float32, device="cuda")
    g = torch.tensor(warm["g"], dtype=torch.float32, device="cuda")
    ot = laue.ot_params(eps, p.distance, c_out, t_b, tol=1e-5, n_max=3000)
    f0, g0, st, rc = laue.laue_sinkhorn(geom, obs, model, ot, f, g, warm["f0"], warm["g0"])
    assert st["converged"] and abs(st["n_iter"] - ref["n_iter"]) <= 2
    # iteration cap: stops exactly at n_max with the warning code
    f = torch.zeros(obs.n, dtype=torch.float32, device="cuda")
    g = torch.zeros(model.n, dtype=torch.float32, device="cuda")
    ot = laue.ot_params(eps, p.distance, c_out, t_b, tol=0.0, n_max=7, chunk=3)
    f0c, g0c, st, rc = laue.laue_sinkhorn(geom, obs, model, ot, f, g)
    assert rc == 1 and st["n_iter"] == 7 and not st["converged"]
    capped = sinkhorn.solve(P, eps, tol=0.0, n_max=7)
    assert g0c == pytest.approx(capped["g0"], abs=1e-3 * eps)


def test_sinkhorn_errors(gpu_lib, prob):
    laue = gpu_lib
    p = prob.preset
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    f = torch.zeros(max(obs.n, 1), dtype=torch.float32, device="cuda")
    g = torch.zeros(max(model.n, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(laue.LaueError) as e:
        laue.laue_sinkhorn(geom, obs, model, laue.ot_params(float("nan"), p.distance, 9.0, 1.0), f, g)
    assert e.value.code == -1
    with pytest.raises(laue.LaueError) as e:
        laue.laue_sinkhorn(geom, obs, model, laue.ot_params(1.0, p.distance, 9.0, 1.0, n_max=0), f, g)
    assert e.value.code == -1
    # T_a = T_b + |I| - |J| < 0 is infeasible: drop all detected spots of the problem
    empty_obs = laue.ObsSpots.from_numpy(np.zeros((0, 2)), np.zeros(prob.geom.n_blocks + 1, np.int64))
    with pytest.raises(laue.LaueError) as e:
        laue.laue_sinkhorn(geom, empty_obs, model, laue.ot_params(1.0, p.distance, 9.0, 0.0), f, g)
    assert e.value.code == -2


def test_sinkhorn_degenerate_blocks(gpu_lib):
    """Blocks without model spots, without detected spots, and a single spot."""
    laue = gpu_lib
    P = _problems.make(ig.TINY, n_rot=3, n_grains=1, seed_shift=5)
    p = P.preset
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    t_b = sinkhorn.default_tb(model.n)
    C = _problems.oracle_costs(P)
    assert any(c.shape[1] == 0 and c.shape[0] > 0 for c in C) or any(c.shape[0] == 0 for c in C)
    eps = 1.0
    Pr = sinkhorn.Problem(C, c_out, 0.0, c_out, t_b)
    ref = sinkhorn.solve(Pr, eps, tol=1e-6, n_max=3000)
    ot = laue.ot_params(eps, p.distance, c_out, t_b, tol=1e-6, n_max=3000)
    f = torch.zeros(max(obs.n, 1), dtype=torch.float32, device="cuda")
    g = torch.zeros(max(model.n, 1), dtype=torch.float32, device="cuda")
    f0, g0, st, rc = laue.laue_sinkhorn(geom, obs, model, ot, f, g)
    assert st["converged"]
    fg = f[:obs.n].cpu().numpy()
    assert np.max(np.abs(fg - ref["f"])) < 1e-3 * max(1.0, np.max(np.abs(ref["f"])))


def test_mstep_matches_oracle(gpu_lib, prob):
    laue = gpu_lib
    p = prob.preset
    eps = 11.1 * p.sigma_mm ** 2
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    t_b = sinkhorn.default_tb(model.n)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    C = _problems.oracle_costs(prob)
    P = sinkhorn.Problem(C, c_out, 0.0, c_out, t_b)
    ref = sinkhorn.solve(P, eps, tol=1e-6, n_max=5000)
    f32 = ig.to_f32_exact(ref["f"])
    g32 = ig.to_f32_exact(ref["g"])
    Qb = sinkhorn.plan_blocks(P, f32, g32, eps)
    p_lab = oem.obs_lab(prob.geom, prob.obs["p12"], prob.obs["block"])
    pairs = oem.grain_pairs(prob.planes, prob.geom, p_lab, prob.obs["offsets"], prob.model, Qb, len(prob.q0))
    k_gn = 2
    q_or, x_or = prob.q0.copy(), prob.x0.copy()
    for _ in range(k_gn):
        for n, pr in enumerate(pairs):
            if pr is not None:
                q_or[n], x_or[n], *_ = mstep.gn_step(pr, q_or[n], x_or[n], prob.geom, p.distance)
    grains = laue.Grains(prob.q0, prob.x0)
    f = torch.tensor(f32, dtype=torch.float32, device="cuda")
    g = torch.tensor(g32, dtype=torch.float32, device="cuda")
    ot = laue.ot_params(eps, p.distance, c_out, t_b)
    laue.laue_mstep(geom, planes, obs, model, ot, f, g, grains, k_gn=k_gn)
    qg, xg = grains.numpy()
    mis = np.degrees(metrics.misorientation(qg, q_or))
    assert np.max(mis) < 1e-3, mis
    assert np.max(np.linalg.norm(xg - x_or, axis=1)) < 2e-3
    # rotations stay unit quaternions, and the step moved the grains
    assert np.allclose(np.linalg.norm(qg, axis=1), 1.0, atol=1e-12)
    assert np.max(np.degrees(metrics.misorientation(qg, prob.q0))) > 1e-3
