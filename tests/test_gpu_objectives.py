"""Plan summaries on the GPU (laue_objectives: mass, inlier and total cost,
entropy, the paper-unit objective) against the oracle's FP64 evaluation of
the same plan (oracle/sinkhorn.py objectives; plan sums for unbalanced OT
and the sparse mask)."""
import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import cost, sinkhorn, sparse
from oracle import unbalanced as ub
from tests import _problems

pytestmark = pytest.mark.gpu

CASES = [("tiny", None, None, 0), ("medium", 4, 60, 0)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-T{c[1]}-N{c[2]}")
def prob(request):
    name, n_rot, n_grains, shift = request.param
    return _problems.make(ig.PRESETS[name], n_rot=n_rot, n_grains=n_grains, seed_shift=shift)


def _dev(a):
    return torch.tensor(np.asarray(a, np.float32), dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("rho", [0, 8])
@pytest.mark.parametrize("eps_scale", [111.0, 3.5])
def test_objectives_match_oracle(gpu_lib, prob, eps_scale, rho):
    laue = gpu_lib
    p = prob.preset
    eps = eps_scale * p.sigma_mm ** 2
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    t_b = sinkhorn.default_tb(model.n)
    if rho:
        prob = _problems.without_tied_rows(prob, rho)
        geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    P = sinkhorn.Problem(_problems.oracle_costs(prob), c_out, 0.0, c_out, t_b)
    if rho:
        P = sparse.masked_problem(P, rho)
    ref = sinkhorn.solve(P, eps, tol=1e-6, n_max=5000)
    f32, g32 = ig.to_f32_exact(ref["f"]), ig.to_f32_exact(ref["g"])
    want = sinkhorn.objectives(P, f32, g32, ref["f0"], ref["g0"], eps, p.sigma_mm, p.distance)
    ot = laue.ot_params(eps, p.distance, c_out, t_b, rho=rho)
    if rho:
        nbr, _, _ = laue.laue_sparse_neighbors(geom, obs, model, ot)
        mo = prob.model["offsets"]
        rows = [sorted((mo[b] + j) for j in np.flatnonzero(np.isfinite(Cb[i]))) for b, Cb in enumerate(P.C)
                for i in range(Cb.shape[0])]
        nbr = nbr.cpu().numpy()
        assert all(sorted(nbr[i, :len(rows[i])].tolist()) == rows[i] for i in range(obs.n))
    got = laue.laue_objectives(geom, obs, model, ot, _dev(f32), _dev(g32), ref["f0"], ref["g0"], p.sigma_mm)
    for k in ("mass", "cost_inlier", "cost_total"):
        assert got[k] == pytest.approx(want[k], rel=2e-5), k
    assert got["entropy"] == pytest.approx(want["entropy"], rel=1e-4, abs=1e-3)
    assert got["sem_objective"] == pytest.approx(want["sem_objective"], rel=1e-5)


def test_objectives_unbalanced_and_errors(gpu_lib, prob):
    laue = gpu_lib
    p = prob.preset
    eps = 11.1 * p.sigma_mm ** 2
    kappa, lam = p.sigma_mm ** 2, 0.4 * p.sigma_mm ** 2
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    C = _problems.oracle_costs(prob)
    ref = ub.solve(C, eps, kappa, lam, tol=1e-6, n_max=5000)
    f32, g32 = ig.to_f32_exact(ref["f"]), ig.to_f32_exact(ref["g"])
    Q = ub.plan_blocks(C, f32, g32, eps)
    mass = sum(q.sum() for q in Q)
    cin = sum(float(np.sum(q * c)) for q, c in zip(Q, C))
    with np.errstate(divide="ignore", invalid="ignore"):
        ent = -sum(float(np.sum(np.where(q > 0, q * np.log(np.where(q > 0, q, 1.0)), 0.0))) for q in Q)
    ot = laue.ot_params(eps, p.distance, 1.0, 0.0, unbalanced_kl=(kappa, lam))
    got = laue.laue_objectives(geom, obs, model, ot, _dev(f32), _dev(g32), 0.0, 0.0, p.sigma_mm)
    assert got["mass"] == pytest.approx(mass, rel=2e-5)
    assert got["cost_inlier"] == pytest.approx(cin, rel=2e-5)
    assert got["cost_total"] == pytest.approx(cin, rel=2e-5)
    assert got["entropy"] == pytest.approx(ent, rel=1e-4, abs=1e-3)
    assert np.isnan(got["sem_objective"])
    with pytest.raises(laue.LaueError) as e:
        laue.laue_objectives(geom, obs, model, ot, _dev(f32), _dev(g32), 0.0, 0.0, 0.0)
    assert e.value.code == -1
