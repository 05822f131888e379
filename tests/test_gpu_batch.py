"""Batched EM: one launch per pass over several independent samples gives
each sample exactly what laue_em gives it alone, and matches the oracle."""
import dataclasses

import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import cost, em as oem, metrics, sinkhorn
from tests import _problems

pytestmark = pytest.mark.gpu


def _sample(laue, preset, n_grains, seed_shift=0):
    p = dataclasses.replace(preset, n_grains=n_grains)
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    q, x = ig.random_grains(p, seed=p.seed + seed_shift)
    obs = laue.laue_simulate(geom, planes, laue.Grains(q, x), p.sigma_mm, p.distance, p.outlier_frac,
                             p.seed + seed_shift)
    q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, p.seed + 17 + seed_shift)
    model = laue.laue_forward_enumerate(geom, planes, laue.Grains(q0, x0), True)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    ot = laue.ot_params(p.eps_start, p.distance, c_out, sinkhorn.default_tb(model.n), tol=1e-5, n_max=2000)
    par = laue.em_params(ot, p.eps_start, p.eps_end, 3, 2)
    return p, geom, planes, obs, model, par, (q0, x0), (q, x)


def test_batched_equals_sequential(gpu_lib):
    laue = gpu_lib
    presets = ig.batching_samples(5)
    samples = [_sample(laue, pr, int(g), k) for k, (pr, g) in enumerate(zip(presets, (12, 30, 7, 20, 16)))]
    # sequential, each alone
    seq = []
    for p, geom, planes, obs, model, par, (q0, x0), _ in samples:
        gr = laue.Grains(q0, x0)
        out = laue.laue_em(geom, planes, obs, model, par, gr)
        seq.append((gr.numpy(), out))
    # one batch
    grains = [laue.Grains(*s[6]) for s in samples]
    rc, outs = laue.laue_em_batched([s[1] for s in samples], [s[2] for s in samples], [s[3] for s in samples],
                                    [s[4] for s in samples], [s[5] for s in samples], grains)
    for k in range(len(samples)):
        (qs, xs), o1 = seq[k]
        qb, xb = grains[k].numpy()
        o2 = outs[k]
        assert np.array_equal(qs, qb) and np.array_equal(xs, xb), k
        for key in ("f", "g", "j_star", "grain", "q_star", "q_out"):
            assert torch.equal(o1[key][:o2[key].numel()], o2[key]), (k, key)
        assert o1["f0"] == o2["f0"] and o1["g0"] == o2["g0"]
        for key in ("n_em_iter", "sinkhorn_iters", "not_converged", "cost_entries", "sinkhorn_passes",
                    "mstep_entries"):
            assert o1[key] == o2[key], (k, key)


def test_batched_matches_oracle(gpu_lib):
    laue = gpu_lib
    probs = [_problems.make(ig.TINY), _problems.make(ig.TINY, seed_shift=5, frac=0.2)]
    args, refs = [], []
    for P in probs:
        p = P.preset
        c_out = cost.c_out(p.sigma_mm, p.distance)
        t_b = sinkhorn.default_tb(len(P.model["m"]))
        eps_list = oem.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
        refs.append(oem.run(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model, P.q0, P.x0,
                            eps_list, c_out, t_b=t_b, k_gn=2, tol=1e-5, n_max=2000))
        geom, planes, obs, model = _problems.gpu_objects(laue, P)
        ot = laue.ot_params(p.eps_start, p.distance, c_out, t_b, tol=1e-5, n_max=2000)
        par = laue.em_params(ot, p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage, k_gn=2)
        args.append((geom, planes, obs, model, par, laue.Grains(P.q0, P.x0)))
    rc, outs = laue.laue_em_batched(*[list(t) for t in zip(*args)])
    for (geom, planes, obs, model, par, gr), ref, o in zip(args, refs, outs):
        qg, xg = gr.numpy()
        assert np.max(np.degrees(metrics.misorientation(qg, ref["q"]))) < 0.01
        assert np.max(np.linalg.norm(xg - ref["x"], axis=1)) < 0.01
        assert o["n_em_iter"] == 20 and o["not_converged"] == 0


@pytest.mark.parametrize("n_grains", [5, 60])
def test_graph_replay_and_tuning_match_direct_launches(gpu_lib, n_grains):
    """The captured chunk is replayed many times per call, with the EM's own
    eager work (evaluation, M-step, polls) between replays; every mode must give
    the direct-launch result bit for bit."""
    laue = gpu_lib
    pr = dataclasses.replace(ig.batching_samples(1)[0], n_rot=30, domega_deg=6.0)
    p, geom, planes, obs, model, par, (q0, x0), _ = _sample(laue, pr, n_grains, 3)
    res = {}
    for launch in (1, 2, 0):
        par.launch = launch
        gr = laue.Grains(q0, x0)
        out = laue.laue_em(geom, planes, obs, model, par, gr)
        res[launch] = (gr.numpy(), out)
    (q1, x1), o1 = res[1]
    assert o1["launch_used"] == 1
    for launch in (2, 0):
        (q, x), o = res[launch]
        assert np.array_equal(q, q1) and np.array_equal(x, x1), launch
        for key in ("f", "g", "j_star", "q_star"):
            assert torch.equal(o[key], o1[key]), (launch, key)
        assert o["sinkhorn_iters"] == o1["sinkhorn_iters"]
    assert res[2][1]["launch_used"] == 2
    assert res[0][1]["launch_used"] in (1, 2)
    # per-stage chunks: fewer polls than iterations
    assert o1["polls"] < o1["sinkhorn_iters"] / 2


def test_batch_with_degenerate_samples(gpu_lib):
    """A sample without model spots (no grains) and one without detected spots
    ride along; every sample still equals its solo run."""
    laue = gpu_lib
    pr = ig.batching_samples(3)
    s0 = _sample(laue, pr[0], 10, 0)
    p, geom, planes, obs, model, par, _, _ = _sample(laue, pr[1], 6, 1)
    empty_g = laue.Grains(np.zeros((0, 4)), np.zeros((0, 3)))
    model_e = laue.laue_forward_enumerate(geom, planes, empty_g, True)
    assert model_e.n == 0
    nb = len(obs.block_off) - 1
    obs_e = laue.ObsSpots.from_numpy(np.zeros((0, 2), np.float32), np.zeros(nb + 1, np.int64))
    samples = [(s0[1], s0[2], s0[3], s0[4], s0[5], laue.Grains(*s0[6])),
               (geom, planes, obs, model_e, par, empty_g),
               (geom, planes, obs_e, model, laue.em_params(laue.ot_params(par.ot.eps, par.ot.distance, par.ot.c_out,
                                                                          float(model.n)),
                                                           par.eps_start, par.eps_end, 3, 2),
                laue.Grains(*_sample(laue, pr[1], 6, 1)[6]))]
    solo = []
    for gm, pl, ob, mo, pa, gr in samples:
        g2 = laue.Grains(*gr.numpy())
        out = laue.laue_em(gm, pl, ob, mo, pa, g2)
        solo.append((g2.numpy(), out))
    rc, outs = laue.laue_em_batched([s[0] for s in samples], [s[1] for s in samples], [s[2] for s in samples],
                                    [s[3] for s in samples], [s[4] for s in samples], [s[5] for s in samples])
    for k, (s, (qx, o1)) in enumerate(zip(samples, solo)):
        qb, xb = s[5].numpy()
        assert np.array_equal(qx[0], qb) and np.array_equal(qx[1], xb), k
        assert o1["sinkhorn_iters"] == outs[k]["sinkhorn_iters"], k


@pytest.mark.parametrize("n_grains", [5, 60])
def test_tile_shapes_match(gpu_lib, n_grains):
    """Two detected (model) spots per lane share each streamed load but keep
    their own arithmetic: every tile shape, fixed or tuned per temperature
    stage, with direct launches or graph replay, gives the one-per-lane result
    bit for bit."""
    laue = gpu_lib
    pr = dataclasses.replace(ig.batching_samples(1)[0], n_rot=30, domega_deg=6.0)
    p, geom, planes, obs, model, par, (q0, x0), _ = _sample(laue, pr, n_grains, 4)
    res = {}
    for tile, launch in ((1, 1), (2, 1), (2, 2), (0, 0)):
        par.tile = tile
        par.launch = launch
        gr = laue.Grains(q0, x0)
        out = laue.laue_em(geom, planes, obs, model, par, gr)
        res[(tile, launch)] = (gr.numpy(), out)
    (q1, x1), o1 = res[(1, 1)]
    assert o1["tile2_solves"] == 0
    assert res[(2, 1)][1]["tile2_solves"] == o1["n_em_iter"]
    for key_run, ((q, x), o) in res.items():
        assert np.array_equal(q, q1) and np.array_equal(x, x1), key_run
        for key in ("f", "g", "j_star", "q_star"):
            assert torch.equal(o[key], o1[key]), (key_run, key)
        assert o["sinkhorn_iters"] == o1["sinkhorn_iters"], key_run


def test_batched_tile_two_equals_solo_tile_one(gpu_lib):
    """Samples batched in the two-per-lane shape equal their solo one-per-lane
    runs (pairs never straddle samples or blocks)."""
    laue = gpu_lib
    presets = ig.batching_samples(4)
    samples = [_sample(laue, pr, int(g), k) for k, (pr, g) in enumerate(zip(presets, (9, 25, 14, 3)))]
    seq = []
    for p, geom, planes, obs, model, par, (q0, x0), _ in samples:
        par.tile = 1
        gr = laue.Grains(q0, x0)
        out = laue.laue_em(geom, planes, obs, model, par, gr)
        seq.append((gr.numpy(), out))
    for s in samples:
        s[5].tile = 2
    grains = [laue.Grains(*s[6]) for s in samples]
    rc, outs = laue.laue_em_batched([s[1] for s in samples], [s[2] for s in samples], [s[3] for s in samples],
                                    [s[4] for s in samples], [s[5] for s in samples], grains)
    for k in range(len(samples)):
        (qs, xs), o1 = seq[k]
        qb, xb = grains[k].numpy()
        assert np.array_equal(qs, qb) and np.array_equal(xs, xb), k
        for key in ("f", "g", "j_star", "q_star"):
            assert torch.equal(o1[key][:outs[k][key].numel()], outs[k][key]), (k, key)
        assert outs[k]["tile2_solves"] == outs[k]["n_em_iter"]
