"""Partial OT E-step on the GPU (Problem A: row and column sums <= 1, total
mass m, no bins; Dykstra's projections from the Gibbs kernel) against the
oracle (oracle/partial.py) on identical FP32 inputs: the dense and sparse
Sinkhorn, the EM, batching, degenerate blocks and the argument checks."""
import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import cost, metrics, sparse
from oracle import em as oem
from oracle import partial as po
from tests import _problems
from tests.test_gpu_unbalanced import _without

pytestmark = pytest.mark.gpu

CASES = [("tiny", None, None, 0), ("medium", 4, 60, 0), ("medium", 3, 100, 1)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-T{c[1]}-N{c[2]}")
def prob(request):
    name, n_rot, n_grains, shift = request.param
    return _problems.make(ig.PRESETS[name], n_rot=n_rot, n_grains=n_grains, seed_shift=shift)


def _solve_gpu(laue, geom, obs, model, ot, fill=0.0):
    # the given potentials are not read: fill them with something else
    f = torch.full((max(obs.n, 1),), fill, dtype=torch.float32, device="cuda")
    g = torch.full((max(model.n, 1),), fill, dtype=torch.float32, device="cuda")
    f0, g0, st, rc = laue.laue_sinkhorn(geom, obs, model, ot, f, g)
    return f, g, f0, g0, st, rc


def _check_against(C, ref, f, g, obs, model, eps):
    fg = f[:obs.n].cpu().numpy().astype(np.float64)
    gg = g[:model.n].cpu().numpy().astype(np.float64)
    # the GPU potentials give a feasible plan of the right mass (FP64 evaluation)
    rows, cols = po.marginals(C, fg, gg, eps)
    assert np.all(rows <= 1 + 2e-4) and np.all(cols <= 1 + 2e-4)
    assert rows.sum() == pytest.approx(ref["mass"], rel=1e-4)
    assert np.all(gg <= 0.0)
    Qg = po.plan_blocks(C, fg, gg, eps)
    Qr = po.plan_blocks(C, ref["f"], ref["g"], eps)
    worst = max((float(np.max(np.abs(a - b))) for a, b in zip(Qg, Qr) if a.size), default=0.0)
    assert worst <= 1e-4, worst
    return fg, gg


@pytest.mark.parametrize("frac", [0.5, 0.9])
@pytest.mark.parametrize("eps_scale", [111.0, 11.1])
def test_partial_sinkhorn_matches_oracle(gpu_lib, prob, eps_scale, frac):
    laue = gpu_lib
    p = prob.preset
    eps = eps_scale * p.sigma_mm ** 2
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    C = _problems.oracle_costs(prob)
    ref = po.solve(C, eps, frac, tol=1e-5, n_max=3000)
    ot = laue.ot_params(eps, p.distance, 1.0, 0.0, tol=1e-5, n_max=3000, partial_frac=frac)
    f, g, f0, g0, st, rc = _solve_gpu(laue, geom, obs, model, ot, fill=3.0)
    assert rc == 0 and st["converged"] and st["err"] <= 1e-5, st
    assert abs(st["n_iter"] - ref["n_iter"]) <= 2, (st, ref["n_iter"])
    assert f0 == -np.inf and g0 == -np.inf
    _check_against(C, ref, f, g, obs, model, eps)


@pytest.mark.parametrize("rho", [8, 32])
def test_partial_sparse_sinkhorn_matches_oracle(gpu_lib, prob, rho):
    laue = gpu_lib
    p = prob.preset
    eps = 11.1 * p.sigma_mm ** 2
    prob = _problems.without_tied_rows(prob, rho)
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    C = sparse.masked_blocks(_problems.oracle_costs(prob), rho)
    ot = laue.ot_params(eps, p.distance, 1.0, 0.0, tol=1e-5, n_max=3000, rho=rho, partial_frac=0.7)
    nbr, _, _ = laue.laue_sparse_neighbors(geom, obs, model, ot)
    nbr = nbr.cpu().numpy()
    mo = prob.model["offsets"]
    want = [sorted((mo[b] + j) for j in np.flatnonzero(np.isfinite(Cb[i]))) for b, Cb in enumerate(C)
            for i in range(Cb.shape[0])]
    assert all(sorted(nbr[i, :len(want[i])].tolist()) == want[i] for i in range(obs.n))
    ref = po.solve(C, eps, 0.7, tol=1e-5, n_max=3000)
    f, g, f0, g0, st, rc = _solve_gpu(laue, geom, obs, model, ot)
    assert rc == 0 and st["converged"] and st["err"] <= 1e-5, st
    assert abs(st["n_iter"] - ref["n_iter"]) <= 2, (st, ref["n_iter"])
    _check_against(C, ref, f, g, obs, model, eps)


def _em_both(laue, P, frac, rho=0):
    p = P.preset
    eps_list = oem.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    ref = oem.run(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model, P.q0, P.x0, eps_list,
                  c_out, k_gn=2, tol=1e-5, n_max=2000, rho=rho or None, partial_frac=frac, record=True)
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    ot = laue.ot_params(p.eps_start, p.distance, c_out, 0.0, tol=1e-5, n_max=2000, rho=rho, partial_frac=frac)
    par = laue.em_params(ot, p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage, k_gn=2)
    gr = laue.Grains(P.q0, P.x0)
    out = laue.laue_em(geom, planes, obs, model, par, gr)
    return ref, out, gr


@pytest.mark.parametrize("rho", [0, 8])
def test_partial_em_matches_oracle(gpu_lib, rho):
    laue = gpu_lib
    P = _problems.make(ig.TINY)
    p = P.preset
    ref, out, gr = _em_both(laue, P, 0.8, rho)
    qg, xg = gr.numpy()
    assert out["code"] == 0 and out["n_em_iter"] == 20 and out["not_converged"] == 0
    assert out["f0"] == -np.inf and out["g0"] == -np.inf
    assert np.max(np.degrees(metrics.misorientation(qg, ref["q"]))) < 0.01
    assert np.max(np.linalg.norm(xg - ref["x"], axis=1)) < 0.01
    assert np.max(np.degrees(metrics.misorientation(qg, P.q_true))) < 0.1
    C, _, _ = oem.build_costs(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model,
                              ref["stats"][-2]["q"], ref["stats"][-2]["x"])     # the last E-step's geometry
    if rho:
        C = sparse.masked_blocks(C, rho)
    js, _, _ = po.hard_assignment(C, ref["f"], ref["g"], p.eps_end)
    assert np.mean(out["j_star"].cpu().numpy() == js) > 0.98


def test_partial_batched_equals_solo(gpu_lib):
    laue = gpu_lib
    from tests.test_gpu_batch import _sample
    presets = ig.batching_samples(3)
    samples = [_sample(laue, pr, int(g), k) for k, (pr, g) in enumerate(zip(presets, (11, 24, 5)))]
    for k, s in enumerate(samples):
        s[5].ot.outlier_model = 2
        s[5].ot.m_frac = 0.6 + 0.1 * k
    seq = []
    for p, geom, planes, obs, model, par, (q0, x0), _ in samples:
        gr = laue.Grains(q0, x0)
        out = laue.laue_em(geom, planes, obs, model, par, gr)
        seq.append((gr.numpy(), out))
    grains = [laue.Grains(*s[6]) for s in samples]
    rc, outs = laue.laue_em_batched([s[1] for s in samples], [s[2] for s in samples], [s[3] for s in samples],
                                    [s[4] for s in samples], [s[5] for s in samples], grains)
    assert rc == 0
    for k in range(len(samples)):
        (qs, xs), o1 = seq[k]
        qb, xb = grains[k].numpy()
        assert np.array_equal(qs, qb) and np.array_equal(xs, xb), k
        for key in ("f", "g", "j_star", "q_star", "q_out"):
            assert torch.equal(o1[key][:outs[k][key].numel()], outs[k][key]), (k, key)


def test_partial_blocks_without_spots_and_argument_checks(gpu_lib):
    laue = gpu_lib
    P0 = _problems.make(ig.TINY)
    both = [b for b in range(P0.geom.n_blocks)
            if np.diff(P0.obs["offsets"])[b] > 0 and np.diff(P0.model["offsets"])[b] > 0]
    P = _without(P0, both[0], both[1])
    p = P.preset
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    C = _problems.oracle_costs(P)
    eps = 11.1 * p.sigma_mm ** 2
    ref = po.solve(C, eps, 0.6, tol=1e-5, n_max=3000)
    ot = laue.ot_params(eps, p.distance, 1.0, 0.0, tol=1e-5, n_max=3000, partial_frac=0.6)
    f, g, f0, g0, st, rc = _solve_gpu(laue, geom, obs, model, ot)
    assert rc == 0 and st["converged"], st
    fg, gg = _check_against(C, ref, f, g, obs, model, eps)
    co = np.concatenate([[0], np.cumsum([c.shape[1] for c in C])])
    assert np.all(gg[co[both[0]]:co[both[0] + 1]] == 0.0)
    for frac in (0.0, 1.5, float("nan")):
        bad = laue.ot_params(eps, p.distance, 1.0, 0.0, partial_frac=frac)
        with pytest.raises(laue.LaueError) as e:
            laue.laue_sinkhorn(geom, obs, model, bad, f, g)
        assert e.value.code == -1, frac
