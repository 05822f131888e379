"""laue_index_batched: every sample of a batch gets what laue_index gives it
alone (grains, assignments and statistics, bit for bit), with the final EMs
in one batch (stage schedules) or one after another (the paper's cooling from
a data-tied first temperature, with the plan-change stop)."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import inputgen as ig

pytestmark = pytest.mark.gpu


def _sample(laue, preset, seed):
    geom = laue.geometry_from_preset(preset)
    planes = laue.laue_planes_cubic(preset.a, preset.centering, preset.n_max)
    q, x = ig.random_grains(preset, seed=seed)
    obs = laue.laue_simulate(geom, planes, laue.Grains(q, x), preset.sigma_mm, preset.distance,
                             preset.outlier_frac, seed)
    return geom, planes, obs


def _no_candidate_sample(laue):
    p = ig.TINY
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    p12 = np.array([[10.0 + t, -20.0] for t in range(p.n_rot)], np.float32)
    off = np.zeros(p.n_rot * 2 + 1, np.int64)
    for t in range(p.n_rot):
        off[2 * t + 1:] += 1
    return geom, planes, laue.ObsSpots.from_numpy(p12, off)


def _presets():
    t = ig.TINY
    return [(t, t.seed), (dataclasses.replace(t, n_rot=18, n_grains=8), t.seed + 1),
            (dataclasses.replace(t, n_grains=3, outlier_frac=0.3), t.seed + 2)]


def _same(solo, batched):
    gs, ss, as_ = solo
    gb, sb, ab = batched
    assert gb.n == gs.n
    assert torch.equal(gb.q[:gb.n], gs.q[:gs.n]) and torch.equal(gb.x[:gb.n], gs.x[:gs.n])
    for k in ("n_candidates", "n_candidates_found", "n_scored", "lbar_entries", "n_picked", "n_prototypes",
              "n_model_spots", "score_pairs"):
        assert sb[k] == ss[k], k
    for k in ("n_em_iter", "sinkhorn_iters", "not_converged", "final_iters_run"):
        assert sb["em"][k] == ss["em"][k], k
    for k in ("sem_objective", "mass", "cost_total"):
        a, b = sb["em"]["objective"][k], ss["em"]["objective"][k]
        assert (math.isnan(a) and math.isnan(b)) or a == b, k
    if as_ is not None:
        for k in as_:
            assert torch.equal(ab[k], as_[k]), k


def test_batched_index_equals_solo_runs(gpu_lib):
    laue = gpu_lib
    items = [(*_sample(laue, p, s), p) for p, s in _presets()]
    items.append((*_no_candidate_sample(laue), ig.TINY))
    pars = [laue.index_params(p, "plain", n_pairs=60, seed=3, n_obs=o.n, n_planes=pl.n)
            for g, pl, o, p in items]
    solo = [laue.laue_index(g, pl, o, par) for (g, pl, o, _), par in zip(items, pars)]
    rc, out = laue.laue_index_batched([it[0] for it in items], [it[1] for it in items], [it[2] for it in items],
                                      pars)
    assert rc == 0
    assert [r[0].n for r in out[:3]] == [s[0].n for s in solo[:3]] and all(s[0].n > 0 for s in solo[:3])
    assert out[3][0].n == 0 and out[3][1]["n_candidates"] == 0
    for s, b in zip(solo, out):
        _same(s, b)


def test_batched_index_paper_cooling_equals_solo_runs(gpu_lib):
    """Data-tied first temperatures give each sample its own number of EM
    temperatures: the EMs run one after another, each as laue_em alone."""
    laue = gpu_lib
    items = [(*_sample(laue, p, s), p) for p, s in _presets()[:2]]
    pars = []
    for g, pl, o, p in items:
        ot = laue.ot_params(1.0, p.distance, laue.c_out_3sigma(p.sigma_mm, p.distance), 0.0)
        em = laue.em_params(ot, 0.0, 2.0 * p.sigma_mm ** 2, 1, 1, eps_cool=0.9, final_iters=6,
                            zeta_tol=1e-3 * math.sqrt(o.n), sigma_mm=p.sigma_mm)
        pars.append(laue.index_params(p, "plain", n_pairs=60, seed=3, n_obs=o.n, n_planes=pl.n, em=em))
    solo = [laue.laue_index(g, pl, o, par) for (g, pl, o, _), par in zip(items, pars)]
    rc, out = laue.laue_index_batched([it[0] for it in items], [it[1] for it in items], [it[2] for it in items],
                                      pars)
    assert rc == 0
    for s, b in zip(solo, out):
        assert s[0].n > 0
        _same(s, b)


def test_batched_index_argument_checks(gpu_lib):
    laue = gpu_lib
    items = [(*_sample(laue, p, s), p) for p, s in _presets()[:2]]
    pars = [laue.index_params(p, "plain", n_pairs=60, seed=3, n_obs=o.n, n_planes=pl.n) for g, pl, o, p in items]
    pars[1].em.ot.rho = 8
    with pytest.raises(laue.LaueError):
        laue.laue_index_batched([it[0] for it in items], [it[1] for it in items], [it[2] for it in items], pars)
