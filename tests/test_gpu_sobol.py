"""Sobol-grid starts on the GPU (Sec. 6.1) against the oracle
(oracle/sobol.py): the kept points and their (q, x), the unrestricted grid,
argument checks, and end-to-end indexing from Sobol starts against the
oracle pipeline with the same starts."""
import math

import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import cost, crystal, em, forward, metrics, pipeline, simulate, sobol

pytestmark = pytest.mark.gpu


def _zone_margin(q):
    q = np.where(q[:, :1] < 0, -q, q)
    a = np.abs(q[:, 1:] / q[:, :1])
    return np.minimum(np.min(sobol.R_FACE - a, axis=1), 1.0 - a.sum(axis=1))


@pytest.mark.parametrize("first", [0, 12345, (1 << 24) + 77])
def test_sobol_starts_match_oracle(gpu_lib, first):
    laue = gpu_lib
    n = 6000
    half = (2.5, 2.0, 1.5)
    qg, xg = laue.laue_sobol_starts(laue.sobol_params(half, first=first), n)
    idx, qo, xo = sobol.starts(first, n, half)
    qg, xg = qg.cpu().numpy(), xg.cpu().numpy()
    if len(qg) != len(qo):
        # only points on the zone's boundary (to rounding) may be decided
        # differently: identify the GPU's points by their positions, check that
        # every disagreement is such a point, and compare the rest
        from scipy.spatial import cKDTree
        pts = sobol.points(first, n)
        allx = (2.0 * pts[:, 3:] - 1.0) * np.asarray(half)
        d, gidx = cKDTree(allx).query(xg)
        assert np.max(d) <= 1e-15
        allq = sobol.mrp_to_quat((2.0 * pts[:, :3] - 1.0) * sobol.MRP_HALF)
        idx = np.asarray(idx) - first
        differ = np.setxor1d(gidx, idx)
        assert np.all(np.abs(_zone_margin(allq[differ])) < 1e-12), differ
        both = np.intersect1d(gidx, idx)
        pos_g = {int(k): r for r, k in enumerate(gidx)}
        pos_o = {int(k): r for r, k in enumerate(idx)}
        rg = np.array([pos_g[int(k)] for k in both])
        ro = np.array([pos_o[int(k)] for k in both])
        qg, xg, qo, xo = qg[rg], xg[rg], qo[ro], xo[ro]
    assert np.max(np.abs(qg - qo)) <= 4e-16 and np.max(np.abs(xg - xo)) <= 1e-15
    assert len(qg) > 0.85 * n


def test_sobol_unrestricted_and_errors(gpu_lib):
    laue = gpu_lib
    q, x = laue.laue_sobol_starts(laue.sobol_params((1.0, 1.0, 1.0), restrict_fz=False), 1000)
    assert q.shape[0] == 1000
    pts = sobol.points(0, 1000)
    assert np.array_equal(x.cpu().numpy(), 2.0 * pts[:, 3:] - 1.0)
    q0, _ = laue.laue_sobol_starts(laue.sobol_params((1.0, 1.0, 1.0)), 0)
    assert q0.shape[0] == 0
    for kw in ({"first": -1}, {"mrp_half": -0.1}, {"mrp_half": float("nan")}):
        with pytest.raises(laue.LaueError) as e:
            laue.laue_sobol_starts(laue.sobol_params((1.0, 1.0, 1.0), **kw), 10)
        assert e.value.code == -1
    with pytest.raises(laue.LaueError):
        laue.laue_sobol_starts(laue.sobol_params((1.0, -1.0, 1.0)), 10)


def _local_sample(laue):
    """Five grains within 4 degrees of the identity and 0.3 mm of the origin
    (tiny geometry), and a Sobol grid over that region."""
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry.from_preset(p)
    rng = np.random.default_rng(11)
    ax = rng.standard_normal((p.n_grains, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    th = np.radians(rng.uniform(1.0, 4.0, p.n_grains))
    q = np.concatenate([np.cos(th / 2)[:, None], np.sin(th / 2)[:, None] * ax], axis=1)
    x = rng.uniform(-0.3, 0.3, (p.n_grains, 3))
    sim = simulate.simulate(pl, q, x, g, p.sigma_mm, p.outlier_frac, p.seed, p.distance)
    p12 = ig.to_f32_exact(sim["p12"])
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    obs = laue.ObsSpots.from_numpy(p12, sim["offsets"])
    return p, pl, g, q, x, sim, p12, geom, planes, obs


def test_index_from_sobol_starts_matches_oracle(gpu_lib):
    laue = gpu_lib
    p, pl, g, qt, xt, sim, p12, geom, planes, obs = _local_sample(laue)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    eps = em.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    mrp_half, half, n_pts = math.tan(math.radians(5.0) / 4), (0.4, 0.4, 0.4), 600
    _, qs, xs = sobol.starts(0, n_pts, half, mrp_half=mrp_half)
    ref = pipeline.index(pl, g, p.distance, p12, sim["offsets"], p.sigma_mm, c_out, eps, 0, 0, starts=(qs, xs))
    par = laue.index_params(p, "sobol", max_candidates=n_pts, n_obs=obs.n, n_planes=planes.n,
                            sobol=laue.sobol_params(half, mrp_half=mrp_half))
    grains, st, asg = laue.laue_index(geom, planes, obs, par)
    assert st["n_candidates"] == len(qs) and st["n_scored"] == len(qs)
    assert st["n_prototypes"] == ref["k"]
    qg, xg = grains.numpy()
    mis = np.degrees(metrics.misorientation(qg[:grains.n][:, None, :], ref["q"][None, :, :]))
    assert np.all(mis.min(axis=1) < 0.01)
    # the Sobol grid over the region finds every grain
    found = np.degrees(metrics.misorientation(qt[:, None, :], qg[None, :grains.n, :])).min(axis=1)
    assert np.all(found < 0.1), found
