"""Pin of the oracle's end-to-end indexing: on noise-free spots without
outliers every indexed grain is a true grain, exactly, and no true grain is
found twice."""
import numpy as np

import inputgen as ig
from oracle import cost, crystal, em, forward, metrics, pipeline, simulate


def test_noise_free_index_is_exact():
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry.from_preset(p)
    q, x = ig.random_grains(p, seed=p.seed)
    sim = simulate.simulate(pl, q, x, g, 0.0, 0.0, p.seed, p.distance)
    p12 = ig.to_f32_exact(sim["p12"])
    c_out = cost.c_out(p.sigma_mm, p.distance)
    eps = em.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    r = pipeline.index(pl, g, p.distance, p12, sim["offsets"], p.sigma_mm, c_out, eps, 60, 3)
    assert r["k"] >= 3
    mis = np.degrees(metrics.misorientation(r["q"][:, None, :], q[None, :, :]))
    best = mis.argmin(axis=1)
    assert len(set(best.tolist())) == r["k"]
    assert np.all(mis.min(axis=1) < 1e-5)
    assert np.all(np.linalg.norm(r["x"] - x[best], axis=1) < 1e-4)
    # the increments drop sharply after the k-th pick
    assert r["gains"][r["k"] - 1] > 1e6 * max(r["gains"][r["k"]:].max(initial=0.0), 1e-300)
