"""GPU parity of the forward model and the simulator against the oracle."""
import numpy as np
import pytest

import inputgen as ig
from oracle import cost, crystal, forward, simulate

pytestmark = pytest.mark.gpu


def _setup(laue, preset, n_rot=None, n_grains=None):
    p = preset
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry(p.n_rot if n_rot is None else n_rot, np.deg2rad(p.domega_deg), p.detectors,
                         p.lam_min, p.lam_max)
    q, x = ig.random_grains(p, n=n_grains)
    geom = laue.make_geometry(g.n_rot, np.deg2rad(p.domega_deg), p.detectors, p.lam_min, p.lam_max)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    return pl, g, q, x, geom, planes


def _compare_sets(V, M, n_det, merge):
    """Index sets equal except items the oracle flags as within the edge margins."""
    o = set(zip(V["t"].tolist(), V["det"].tolist(), V["n"].tolist(), V["m"].tolist()))
    g = set(zip((M["block"] // n_det).tolist(), (M["block"] % n_det).tolist(), M["grain"].tolist(),
                M["plane"].tolist()))
    flagged = {k for k, f in zip(zip(V["t"].tolist(), V["det"].tolist(), V["n"].tolist(),
                                     V["m"].tolist()), V["flag"]) if f}
    flagged |= {(t, d, n, m) for (n, t, m, d) in V["near_edge"]}
    gflag = {k for k, f in zip(zip((M["block"] // n_det).tolist(), (M["block"] % n_det).tolist(),
                                   M["grain"].tolist(), M["plane"].tolist()), M["flags"]) if f}
    diff = (o ^ g) - flagged - gflag
    assert not diff, f"{len(diff)} unflagged differences, e.g. {sorted(diff)[:5]}"
    return o & g


@pytest.mark.parametrize("name,n_rot,n_grains,merge", [("tiny", None, None, True),
                                                       ("tiny", None, None, False),
                                                       ("medium", None, None, True),
                                                       ("medium", 7, 40, False),
                                                       ("stress", 5, 60, True)])
def test_enumerate_matches_oracle(gpu_lib, name, n_rot, n_grains, merge):
    laue = gpu_lib
    pl, g, q, x, geom, planes = _setup(laue, ig.PRESETS[name], n_rot, n_grains)
    V = forward.enumerate_visible(pl, q, x, g, merge_harmonics=merge)
    M = laue.laue_forward_enumerate(geom, planes, laue.Grains(q, x), merge).numpy()
    common = _compare_sets(V, M, g.n_det, merge)
    assert len(common) > 0.99 * len(V["m"])
    # order (t, d, n, m) and block offsets
    key = M["block"].astype(np.int64) * 10**9 + M["grain"].astype(np.int64) * 10**4 + M["plane"]
    assert np.all(np.diff(key) > 0)
    assert np.array_equal(M["block_off"], np.concatenate([[0], np.cumsum(np.bincount(M["block"], minlength=g.n_blocks))]))
    # positions and wavelengths of common items
    idx = {k: i for i, k in enumerate(zip(V["t"].tolist(), V["det"].tolist(), V["n"].tolist(), V["m"].tolist()))}
    gi, oi = [], []
    for j, k in enumerate(zip((M["block"] // g.n_det).tolist(), (M["block"] % g.n_det).tolist(),
                              M["grain"].tolist(), M["plane"].tolist())):
        if k in idx:
            gi.append(j)
            oi.append(idx[k])
    gi, oi = np.array(gi), np.array(oi)
    assert np.max(np.abs(M["s1"][gi] - V["s12"][oi, 0])) < 2e-3
    assert np.max(np.abs(M["s2"][gi] - V["s12"][oi, 1])) < 2e-3
    assert np.max(np.abs(M["lam"][gi] - V["lam"][oi]) / V["lam"][oi]) < 1e-6
    ev = forward.eval_fixed(pl, q, x, g, V["m"][oi], V["n"][oi], V["t"][oi], V["det"][oi])
    vl = cost.v_local(g, V["det"][oi], ev["v"])
    for c, col in enumerate(("vn", "v1", "v2")):
        assert np.max(np.abs(M[col][gi] - vl[:, c])) < 2e-3


def test_enumerate_empty_and_capacity(gpu_lib):
    laue = gpu_lib
    pl, g, q, x, geom, planes = _setup(laue, ig.TINY)
    M = laue.laue_forward_enumerate(geom, planes, laue.Grains(np.zeros((0, 4)), np.zeros((0, 3))))
    assert M.n == 0 and np.all(M.block_off == 0)


def test_eval_matches_oracle(gpu_lib):
    laue = gpu_lib
    pl, g, q, x, geom, planes = _setup(laue, ig.MEDIUM, 9, 30)
    S = forward.enumerate_visible(pl, q, x, g)
    q2, x2 = ig.perturb_grains(q, x, 0.7, 0.4, 5)
    M = laue.ModelSpots.from_arrays(g.n_blocks, forward.block_offsets(S["block"], g.n_blocks),
                                    S["m"], S["n"], S["block"])
    laue.laue_forward_eval(geom, planes, laue.Grains(q2, x2), M)
    Mg = M.numpy()
    ev = forward.eval_fixed(pl, q2, x2, g, S["m"], S["n"], S["t"], S["det"])
    vl = cost.v_local(g, S["det"], ev["v"])
    assert np.max(np.abs(Mg["s1"] - ev["s12"][:, 0])) < 2e-3
    assert np.max(np.abs(Mg["s2"] - ev["s12"][:, 1])) < 2e-3
    for c, col in enumerate(("vn", "v1", "v2")):
        assert np.max(np.abs(Mg[col] - vl[:, c])) < 2e-3


@pytest.mark.parametrize("name,n_rot,n_grains", [("tiny", None, None), ("medium", 6, 50)])
def test_simulate_matches_oracle(gpu_lib, name, n_rot, n_grains):
    laue = gpu_lib
    p = ig.PRESETS[name]
    pl, g, q, x, geom, planes = _setup(laue, p, n_rot, n_grains)
    sim = simulate.simulate(pl, q, x, g, p.sigma_mm, p.outlier_frac, p.seed, p.distance)
    ob = laue.laue_simulate(geom, planes, laue.Grains(q, x), p.sigma_mm, p.distance, p.outlier_frac, p.seed)
    assert np.array_equal(ob.block_off, sim["offsets"])
    n = ob.n
    p1 = ob.p1[:n].cpu().numpy()
    p2 = ob.p2[:n].cpu().numpy()
    assert np.array_equal(ob.grain[:n].cpu().numpy(), sim["grain"])
    assert np.array_equal(ob.plane[:n].cpu().numpy(), sim["plane"])
    assert np.max(np.abs(p1 - sim["p12"][:, 0])) < 1e-3
    assert np.max(np.abs(p2 - sim["p12"][:, 1])) < 1e-3
