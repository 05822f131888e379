"""Unbalanced OT E-step on the GPU (Problem B: KL-relaxed marginals, no bins)
against the oracle (oracle/unbalanced.py) on identical FP32 inputs: the
dense and sparse Sinkhorn, the hard assignment, the EM, batching, and the
argument checks."""
import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import cost, metrics, sparse
from oracle import em as oem
from oracle import unbalanced as ub
from tests import _problems

pytestmark = pytest.mark.gpu

CASES = [("tiny", None, None, 0), ("medium", 4, 60, 0), ("medium", 3, 100, 1)]
# (kappa, lambda) in units of 2 sigma^2 (the paper's log-likelihood units), spanning its range
KL = [(0.5, 0.1), (1.0, 1.0), (0.02, 0.3)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-T{c[1]}-N{c[2]}")
def prob(request):
    name, n_rot, n_grains, shift = request.param
    return _problems.make(ig.PRESETS[name], n_rot=n_rot, n_grains=n_grains, seed_shift=shift)


def _kl_mm2(p, kl):
    s2 = 2.0 * p.sigma_mm ** 2
    return kl[0] * s2, kl[1] * s2


def _solve_gpu(laue, geom, obs, model, ot):
    f = torch.zeros(max(obs.n, 1), dtype=torch.float32, device="cuda")
    g = torch.zeros(max(model.n, 1), dtype=torch.float32, device="cuda")
    f0, g0, st, rc = laue.laue_sinkhorn(geom, obs, model, ot, f, g)
    return f, g, f0, g0, st, rc


def _check_against(C, ref, f, g, obs, model, eps, kappa, lam):
    fg = f[:obs.n].cpu().numpy().astype(np.float64)
    gg = g[:model.n].cpu().numpy().astype(np.float64)
    # the GPU potentials satisfy the first-order marginal conditions, evaluated in FP64
    rows, cols = ub.marginals(C, fg, gg, eps)
    live = rows > 1e-30
    assert np.max(np.abs(rows[live] - np.exp(-fg[live] / kappa))) < 2e-4
    live = cols > 1e-30
    assert np.max(np.abs(cols[live] - np.exp(-gg[live] / lam))) < 2e-4
    Qg = ub.plan_blocks(C, fg, gg, eps)
    Qr = ub.plan_blocks(C, ref["f"], ref["g"], eps)
    worst = max((float(np.max(np.abs(a - b))) for a, b in zip(Qg, Qr) if a.size), default=0.0)
    assert worst <= 1e-4, worst
    return fg, gg


@pytest.mark.parametrize("kl", KL, ids=lambda k: f"k{k[0]}-l{k[1]}")
@pytest.mark.parametrize("eps_scale", [111.0, 11.1])
def test_unbalanced_sinkhorn_matches_oracle(gpu_lib, prob, eps_scale, kl):
    laue = gpu_lib
    p = prob.preset
    eps = eps_scale * p.sigma_mm ** 2
    kappa, lam = _kl_mm2(p, kl)
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    C = _problems.oracle_costs(prob)
    ref = ub.solve(C, eps, kappa, lam, tol=1e-5, n_max=3000)
    # bin costs and T_b are not read under unbalanced OT
    ot = laue.ot_params(eps, p.distance, 1.0, 0.0, tol=1e-5, n_max=3000, unbalanced_kl=(kappa, lam))
    f, g, f0, g0, st, rc = _solve_gpu(laue, geom, obs, model, ot)
    assert rc == 0 and st["converged"] and st["err"] <= 1e-5, st
    assert abs(st["n_iter"] - ref["n_iter"]) <= 2, (st, ref["n_iter"])
    assert f0 == -np.inf and g0 == -np.inf
    _check_against(C, ref, f, g, obs, model, eps, kappa, lam)


@pytest.mark.parametrize("rho", [8, 32])
def test_unbalanced_sparse_sinkhorn_matches_oracle(gpu_lib, prob, rho):
    laue = gpu_lib
    p = prob.preset
    eps = 11.1 * p.sigma_mm ** 2
    kappa, lam = _kl_mm2(p, (0.5, 0.1))
    prob = _problems.without_tied_rows(prob, rho)
    geom, planes, obs, model = _problems.gpu_objects(laue, prob)
    C = sparse.masked_blocks(_problems.oracle_costs(prob), rho)
    ot = laue.ot_params(eps, p.distance, 1.0, 0.0, tol=1e-5, n_max=3000, rho=rho, unbalanced_kl=(kappa, lam))
    nbr, _, _ = laue.laue_sparse_neighbors(geom, obs, model, ot)
    nbr = nbr.cpu().numpy()
    mo = prob.model["offsets"]
    want = [sorted((mo[b] + j) for j in np.flatnonzero(np.isfinite(Cb[i]))) for b, Cb in enumerate(C)
            for i in range(Cb.shape[0])]
    assert all(sorted(nbr[i, :len(want[i])].tolist()) == want[i] for i in range(obs.n))
    ref = ub.solve(C, eps, kappa, lam, tol=1e-5, n_max=3000)
    f, g, f0, g0, st, rc = _solve_gpu(laue, geom, obs, model, ot)
    assert rc == 0 and st["converged"] and st["err"] <= 1e-5, st
    assert abs(st["n_iter"] - ref["n_iter"]) <= 2, (st, ref["n_iter"])
    fg, gg = _check_against(C, ref, f, g, obs, model, eps, kappa, lam)
    # model spots no detected spot keeps have potential 0 on both sides
    kept = np.zeros(model.n, bool)
    kept[nbr[nbr >= 0]] = True
    assert np.all(gg[~kept] == 0.0) and np.all(ref["g"][~kept] == 0.0)


def _em_both(laue, P, kl, rho=0, k_gn=2):
    p = P.preset
    kappa, lam = _kl_mm2(p, kl)
    eps_list = oem.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    ref = oem.run(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model, P.q0, P.x0, eps_list,
                  c_out, k_gn=k_gn, tol=1e-5, n_max=2000, rho=rho or None, unbalanced_kl=(kappa, lam), record=True)
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    ot = laue.ot_params(p.eps_start, p.distance, c_out, 0.0, tol=1e-5, n_max=2000, rho=rho,
                        unbalanced_kl=(kappa, lam))
    par = laue.em_params(ot, p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage, k_gn=k_gn)
    gr = laue.Grains(P.q0, P.x0)
    out = laue.laue_em(geom, planes, obs, model, par, gr)
    return ref, out, gr, (kappa, lam)


@pytest.mark.parametrize("rho", [0, 8])
def test_unbalanced_em_matches_oracle(gpu_lib, rho):
    laue = gpu_lib
    P = _problems.make(ig.TINY)
    p = P.preset
    ref, out, gr, (kappa, lam) = _em_both(laue, P, (0.5, 0.5), rho)
    qg, xg = gr.numpy()
    assert out["code"] == 0 and out["n_em_iter"] == 20 and out["not_converged"] == 0
    assert out["f0"] == -np.inf and out["g0"] == -np.inf
    assert np.max(np.degrees(metrics.misorientation(qg, ref["q"]))) < 0.01
    assert np.max(np.linalg.norm(xg - ref["x"], axis=1)) < 0.01
    assert np.max(np.degrees(metrics.misorientation(qg, P.q_true))) < 0.1
    # hard assignments agree with the oracle's at its final state (near-ties aside)
    C, _, _ = oem.build_costs(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model,
                              ref["stats"][-2]["q"], ref["stats"][-2]["x"])     # the last E-step's geometry
    if rho:
        C = sparse.masked_blocks(C, rho)
    js, _, _ = ub.hard_assignment(C, ref["f"], ref["g"], p.eps_end)
    jg = out["j_star"].cpu().numpy()
    assert np.mean(jg == js) > 0.98
    # spots assigned to a model spot mostly go to their true grain
    lab = P.obs["grain"]
    gs = out["grain"].cpu().numpy()
    matched = (lab >= 0) & (gs >= 0)
    assert matched.sum() > 0.5 * (lab >= 0).sum()
    assert np.mean(gs[matched] == lab[matched]) > 0.95


@pytest.mark.parametrize("rho", [0, 8])
def test_unbalanced_assignment_at_gpu_potentials(gpu_lib, rho):
    """The assignment kernel's decisions equal the oracle's rule evaluated on
    the GPU's own final potentials, wherever the deciding margin exceeds the
    FP32 rounding of the quantities compared."""
    laue = gpu_lib
    P = _problems.make(ig.PRESETS["medium"], n_rot=4, n_grains=60)
    p = P.preset
    # one stage, one iteration, no M-step: the assignment is taken at the E-step geometry,
    # which is then the starting grains
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    kappa, lam = _kl_mm2(p, (1.0, 0.2))
    ot = laue.ot_params(p.eps_end, p.distance, 1.0, 0.0, tol=1e-5, n_max=3000, rho=rho, unbalanced_kl=(kappa, lam))
    par = laue.em_params(ot, p.eps_end, p.eps_end, 1, 1, k_gn=0)
    g0r = laue.Grains(P.q0, P.x0)
    o = laue.laue_em(geom, planes, obs, model, par, g0r)
    assert o["code"] == 0
    C, _, _ = oem.build_costs(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model, P.q0, P.x0)
    if rho:
        C = sparse.masked_blocks(C, rho)
    fg = o["f"][:obs.n].cpu().numpy().astype(np.float64)
    gg = o["g"][:model.n].cpu().numpy().astype(np.float64)
    js, qs, qo = ub.hard_assignment(C, fg, gg, p.eps_end)
    jg = o["j_star"].cpu().numpy()
    qog = o["q_out"].cpu().numpy()
    assert np.max(np.abs(qog - qo)) < 1e-3
    # decisive margin: best entry vs runner-up and vs the deficit
    Q = ub.plan_blocks(C, fg, gg, p.eps_end)
    ro = np.concatenate([[0], np.cumsum([c.shape[0] for c in C])])
    clear = np.zeros(obs.n, bool)
    for b, q in enumerate(Q):
        for i in range(q.shape[0]):
            row = np.sort(np.concatenate([q[i], [qo[ro[b] + i]]]))[::-1]
            clear[ro[b] + i] = len(row) < 2 or row[0] - row[1] > 1e-3 * max(row[0], 1e-30) + 1e-6
    assert clear.mean() > 0.9
    assert np.array_equal(jg[clear], js[clear])


def test_unbalanced_batched_equals_solo(gpu_lib):
    laue = gpu_lib
    from tests.test_gpu_batch import _sample
    presets = ig.batching_samples(3)
    samples = [_sample(laue, pr, int(g), k) for k, (pr, g) in enumerate(zip(presets, (11, 24, 5)))]
    for k, s in enumerate(samples):
        s2 = 2.0 * s[0].sigma_mm ** 2
        s[5].ot.outlier_model = 1
        s[5].ot.kappa, s[5].ot.lam = (0.5 + 0.2 * k) * s2, 0.3 * s2
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
        assert o1["sinkhorn_iters"] == outs[k]["sinkhorn_iters"]


def test_unbalanced_argument_checks_and_degenerate(gpu_lib):
    laue = gpu_lib
    P = _problems.make(ig.TINY)
    p = P.preset
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    eps = 11.1 * p.sigma_mm ** 2
    f = torch.zeros(max(obs.n, 1), dtype=torch.float32, device="cuda")
    g = torch.zeros(max(model.n, 1), dtype=torch.float32, device="cuda")
    for kl, model_id in (((0.0, 1.0), 1), ((1.0, -1.0), 1), ((float("inf"), 1.0), 1), ((1.0, 1.0), 2)):
        ot = laue.ot_params(eps, p.distance, 1.0, 0.0, unbalanced_kl=kl)
        ot.outlier_model = model_id
        with pytest.raises(laue.LaueError) as e:
            laue.laue_sinkhorn(geom, obs, model, ot, f, g)
        assert e.value.code == -1, (kl, model_id)
    # non-finite bin potentials are refused under the outlier row and column only
    ot = laue.ot_params(eps, p.distance, cost.c_out(p.sigma_mm, p.distance), 10.0)
    with pytest.raises(laue.LaueError) as e:
        laue.laue_sinkhorn(geom, obs, model, ot, f, g, f0=-np.inf)
    assert e.value.code == -1
    ot = laue.ot_params(eps, p.distance, 1.0, 0.0, unbalanced_kl=(1.0, 1.0))
    assert laue.laue_sinkhorn(geom, obs, model, ot, f, g, f0=-np.inf, g0=-np.inf)[3] == 0
    # no detected spots: feasible without bins; every column is empty and gets potential 0
    empty_obs = laue.ObsSpots.from_numpy(np.zeros((0, 2)), np.zeros(P.geom.n_blocks + 1, np.int64))
    g.fill_(3.0)
    f0, g0, st, rc = laue.laue_sinkhorn(geom, empty_obs, model, ot, f, g)
    assert rc == 0 and st["converged"]
    assert torch.all(g[:model.n] == 0.0)


def _without(P, obs_block, model_block):
    """P with the detected spots of one block and the model spots of another removed."""
    import dataclasses
    off, mo = P.obs["offsets"], P.model["offsets"]
    ki = np.ones(off[-1], bool)
    ki[off[obs_block]:off[obs_block + 1]] = False
    kj = np.ones(mo[-1], bool)
    kj[mo[model_block]:mo[model_block + 1]] = False
    obs = {k: (v[ki] if isinstance(v, np.ndarray) and len(v) == off[-1] else v) for k, v in P.obs.items()}
    obs["offsets"] = np.concatenate([[0], np.cumsum(np.diff(off) * (np.arange(len(off) - 1) != obs_block))])
    model = {k: (v[kj] if isinstance(v, np.ndarray) and len(v) == mo[-1] else v) for k, v in P.model.items()}
    model["offsets"] = np.concatenate([[0], np.cumsum(np.diff(mo) * (np.arange(len(mo) - 1) != model_block))])
    return dataclasses.replace(P, obs=obs, model=model, s12=P.s12[kj], vloc=P.vloc[kj])


def test_unbalanced_blocks_without_spots(gpu_lib):
    """A block whose model spots are removed (its rows get potential 0) and
    one whose detected spots are removed (its columns get 0)."""
    laue = gpu_lib
    P0 = _problems.make(ig.TINY)
    both = [b for b in range(P0.geom.n_blocks)
            if np.diff(P0.obs["offsets"])[b] > 0 and np.diff(P0.model["offsets"])[b] > 0]
    P = _without(P0, both[0], both[1])
    p = P.preset
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    C = _problems.oracle_costs(P)
    assert C[both[0]].shape[0] == 0 and C[both[0]].shape[1] > 0
    assert C[both[1]].shape[1] == 0 and C[both[1]].shape[0] > 0
    eps = 11.1 * p.sigma_mm ** 2
    kappa, lam = _kl_mm2(p, (0.5, 0.1))
    ref = ub.solve(C, eps, kappa, lam, tol=1e-5, n_max=3000)
    ot = laue.ot_params(eps, p.distance, 1.0, 0.0, tol=1e-5, n_max=3000, unbalanced_kl=(kappa, lam))
    f, g, f0, g0, st, rc = _solve_gpu(laue, geom, obs, model, ot)
    assert rc == 0 and st["converged"], st
    assert abs(st["n_iter"] - ref["n_iter"]) <= 2, (st, ref["n_iter"])
    fg, gg = _check_against(C, ref, f, g, obs, model, eps, kappa, lam)
    ro = np.concatenate([[0], np.cumsum([c.shape[0] for c in C])])
    co = np.concatenate([[0], np.cumsum([c.shape[1] for c in C])])
    b0, b1 = both[0], both[1]
    assert np.all(gg[co[b0]:co[b0 + 1]] == 0.0)
    assert np.all(fg[ro[b1]:ro[b1 + 1]] == 0.0)
