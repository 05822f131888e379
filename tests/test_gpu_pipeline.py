"""GPU parity of end-to-end indexing (laue_index) against the oracle
pipeline, plain and learned modes, and recovery on a larger workload."""
import math

import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import candidates, cost, crystal, em, forward, metrics, mlp as omlp, pipeline, proposal, simulate

pytestmark = pytest.mark.gpu


def _tiny(laue, sigma=None, frac=None):
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry.from_preset(p)
    q, x = ig.random_grains(p, seed=p.seed)
    sim = simulate.simulate(pl, q, x, g, p.sigma_mm if sigma is None else sigma,
                            p.outlier_frac if frac is None else frac, p.seed, p.distance)
    p12 = ig.to_f32_exact(sim["p12"])
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    obs = laue.ObsSpots.from_numpy(p12, sim["offsets"])
    c_out = cost.c_out(p.sigma_mm, p.distance)
    eps = em.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    return p, pl, g, q, x, sim, p12, geom, planes, obs, c_out, eps


def _match(qa, xa, qb, xb):
    """Pairs (i, j) of grains of a and b closer than 0.5 deg, greedily."""
    if len(qa) == 0 or len(qb) == 0:
        return []
    mis = np.degrees(metrics.misorientation(qa[:, None, :], qb[None, :, :]))
    out, used = [], set()
    for i in np.argsort(mis.min(axis=1)):
        j = int(np.argmin(np.where([k in used for k in range(len(qb))], np.inf, mis[i])))
        if mis[i, j] < 0.5 and j not in used:
            used.add(j)
            out.append((int(i), j, mis[i, j], np.linalg.norm(xa[i] - xb[j])))
    return out


def test_index_plain_matches_oracle(gpu_lib):
    laue = gpu_lib
    p, pl, g, q, x, sim, p12, geom, planes, obs, c_out, eps = _tiny(laue)
    ref = pipeline.index(pl, g, p.distance, p12, sim["offsets"], p.sigma_mm, c_out, eps, 60, 3)
    par = laue.index_params(p, "plain", n_pairs=60, seed=3, n_obs=obs.n, n_planes=planes.n)
    grains, st, asg = laue.laue_index(geom, planes, obs, par)
    print("oracle k", ref["k"], "gpu", st)
    assert st["n_candidates"] == len(ref["candidates"]["q"]) or \
        abs(st["n_candidates"] - len(ref["candidates"]["q"])) <= 2e-3 * len(ref["candidates"]["q"])
    assert st["n_prototypes"] == ref["k"]
    qg, xg = grains.numpy()
    m = _match(qg[:grains.n], xg[:grains.n], ref["q"], ref["x"])
    assert len(m) == ref["k"]
    for i, j, mis, dx in m:
        assert mis < 0.01 and dx < 2e-3, (mis, dx)
    # assignments: outliers or grains of the result
    gr = asg["grain"].cpu().numpy()
    assert np.all((gr >= -1) & (gr < grains.n))


def test_index_learned_matches_oracle(gpu_lib):
    laue = gpu_lib
    p, pl, g, q, x, sim, p12, geom, planes, obs, c_out, eps = _tiny(laue)
    prm = omlp.init(seed=9)
    net = laue.Mlp(params=laue.Mlp.pack(prm))
    # oracle ranking: features of the oracle candidates, the oracle network
    cand = candidates.generate(pl, g, p12, sim["offsets"], 60, 3)
    t_pair = (np.searchsorted(sim["offsets"], cand["a"], side="right") - 1) // g.n_det
    sup, _ = proposal.support(pl, g, p12, sim["offsets"], cand["q"], t_pair, 1.0, len(pl["d"]))
    feat = np.concatenate([cand["feat"], sup], axis=1).astype(np.float32).astype(np.float64)
    rank, _ = omlp.forward(prm, feat)
    ref = pipeline.index(pl, g, p.distance, p12, sim["offsets"], p.sigma_mm, c_out, eps, 60, 3, ranking=rank,
                         top_frac=0.5)
    par = laue.index_params(p, "learned", n_pairs=60, seed=3, mlp=net, top_frac=0.5, n_obs=obs.n,
                            n_planes=planes.n)
    grains, st, _ = laue.laue_index(geom, planes, obs, par)
    assert st["n_scored"] == math.ceil(0.5 * st["n_candidates"])
    assert abs(st["n_prototypes"] - ref["k"]) <= 1
    qg, xg = grains.numpy()
    m = _match(qg[:grains.n], xg[:grains.n], ref["q"], ref["x"])
    assert len(m) >= min(grains.n, ref["k"]) - 1
    for i, j, mis, dx in m:
        assert mis < 0.01 and dx < 2e-3, (mis, dx)


def test_index_recovers_medium_grains(gpu_lib):
    laue = gpu_lib
    p = ig.MEDIUM
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    q, x = ig.random_grains(p, seed=p.seed)
    truth = laue.Grains(q, x)
    obs = laue.laue_simulate(geom, planes, truth, p.sigma_mm, p.distance, p.outlier_frac, p.seed)
    par = laue.index_params(p, "plain", n_pairs=4096, seed=1, n_obs=obs.n, n_planes=planes.n)
    grains, st, asg = laue.laue_index(geom, planes, obs, par)
    print(st)
    qg, xg = grains.numpy()
    rec, _ = metrics.match_grains(qg[:grains.n], xg[:grains.n], q, x)
    print("recovered", rec, "of", len(q), "prototypes", grains.n)
    assert rec >= 0.9 * len(q)


def test_index_without_candidates(gpu_lib):
    """Spots that pair into no hypothesis (one spot per rotation) index to no
    grain, without error."""
    laue = gpu_lib
    p = ig.TINY
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    nb = p.n_rot * 2
    p12 = np.array([[10.0 + t, -20.0] for t in range(p.n_rot)], np.float32)
    off = np.zeros(nb + 1, np.int64)
    for t in range(p.n_rot):
        off[2 * t + 1:] += 1          # one spot on the transmission detector of every rotation
    obs = laue.ObsSpots.from_numpy(p12, off)
    par = laue.index_params(p, "plain", n_pairs=64, seed=1, n_obs=obs.n, n_planes=planes.n)
    grains, st, asg = laue.laue_index(geom, planes, obs, par)
    assert st["n_candidates"] == 0 and grains.n == 0 and st["n_prototypes"] == 0
