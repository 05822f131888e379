"""Pins of the oracle forward model against closed forms and invariants."""
import numpy as np
import pytest

import inputgen as ig
from oracle import crystal, forward, simulate

A = 2.87


def _geom(n_rot=1, domega=0.0, lam=(1.0, 4.0)):
    return forward.Geometry(n_rot, domega, ig.MEDIUM.detectors, *lam)


def _ident():
    return np.array([[1.0, 0, 0, 0]]), np.zeros((1, 3))


def test_worked_example_411_and_200():
    # R = I, x = 0, Gamma = I: lambda = 2 a h / N, r = e - 2 (h/sqrt N) (h,k,l)/sqrt N
    pl = crystal.cubic_planes(A, "I", 30)
    idx = {tuple(v): i for i, v in enumerate(pl["hkl"].tolist())}
    q, x = _ident()
    V = forward.enumerate_visible(pl, q, x, _geom(), merge_harmonics=False)
    hit = {int(m): k for k, m in enumerate(V["m"])}
    k = hit[idx[(4, 1, 1)]]
    assert V["lam"][k] == pytest.approx(4 * A / 9, abs=1e-12)
    assert np.allclose(V["r"][k], [-7 / 9, -4 / 9, -4 / 9], atol=1e-14)
    assert V["det"][k] == 1 and V["tau"][k] == pytest.approx(1350 / 7)
    assert np.allclose(V["s"][k], [-150, -600 / 7, -600 / 7], atol=1e-10)
    assert np.allclose(V["s12"][k], [-600 / 7, -600 / 7], atol=1e-10)
    k = hit[idx[(2, 0, 0)]]
    assert V["lam"][k] == pytest.approx(A)
    assert np.allclose(V["r"][k], [-1, 0, 0]) and np.allclose(V["s"][k], [-150, 0, 0])
    # (-4,1,1) has negative lambda: never visible
    assert idx[(-4, 1, 1)] not in hit


def _sample(seed=3, n=6, n_rot=8):
    pl = crystal.cubic_planes(A, "I", 30)
    g = _geom(n_rot, np.deg2rad(7.0))
    rng = np.random.default_rng(seed)
    q = ig.random_quaternions(rng, n)
    x = ig.random_positions(rng, n, 2.5, 5.0)
    return pl, g, q, x


def test_bragg_and_ray_invariants():
    pl, g, q, x = _sample()
    V = forward.enumerate_visible(pl, q, x, g, merge_harmonics=False)
    assert len(V["m"]) > 100
    r = V["r"]
    assert np.allclose(np.linalg.norm(r, axis=1), 1.0)
    # Bragg: lambda = 2 d sin(theta) with cos(2 theta) = r.e
    sin_t = np.sqrt((1.0 - r[:, 0]) / 2.0)
    assert np.allclose(V["lam"], 2.0 * pl["d"][V["m"]] * sin_t, rtol=1e-12)
    # r - e is parallel to the rotated plane normal u
    R = crystal.quat_to_R(q)
    u = np.einsum("jab,jbc,jc->ja", g.G[V["t"]], R[V["n"]], pl["w"][V["m"]])
    assert np.allclose(np.cross(r - [1, 0, 0], u), 0.0, atol=1e-12)
    assert np.all((V["lam"] >= 1.0) & (V["lam"] <= 4.0))
    # spots lie on their detector plane, within the square, in front of the grain
    assert np.all(V["tau"] > 0)
    assert np.allclose(V["s"][:, 0], np.where(V["det"] == 0, 150.0, -150.0))
    assert np.all(np.max(np.abs(V["s12"]), axis=1) < 100.0)
    # at most one of +-hkl per (grain, rotation)
    hkl = {tuple(v): i for i, v in enumerate(pl["hkl"].tolist())}
    neg = np.array([hkl[tuple(-x for x in v)] for v in pl["hkl"].tolist()])
    keys = set(zip(V["n"].tolist(), V["t"].tolist(), V["m"].tolist()))
    for n_, t_, m_ in keys:
        assert (n_, t_, int(neg[m_])) not in keys


def test_cubic_symmetry_invariance():
    pl, g, q, x = _sample(seed=5, n=3, n_rot=4)
    S = forward.enumerate_visible(pl, q, x, g)
    for Sm in crystal.cubic_group()[[3, 11, 17]]:
        qs = np.array([crystal.R_to_quat(R @ Sm) for R in crystal.quat_to_R(q)])
        S2 = forward.enumerate_visible(pl, qs, x, g)
        a = np.sort(np.round(np.c_[S["t"], S["det"], S["n"], S["s12"]], 8), axis=0)
        b = np.sort(np.round(np.c_[S2["t"], S2["det"], S2["n"], S2["s12"]], 8), axis=0)
        assert np.array_equal(a, b)


def test_rotation_composition():
    # grain (R, x) seen at rotation t == grain (Gamma_t R, Gamma_t x) seen at omega = 0
    pl, g, q, x = _sample(seed=7, n=2, n_rot=5)
    S = forward.enumerate_visible(pl, q, x, g)
    t = 3
    R = crystal.quat_to_R(q)
    q2 = np.array([crystal.R_to_quat(g.G[t] @ Rn) for Rn in R])
    x2 = x @ g.G[t].T
    g0 = _geom(1, 0.0)
    S2 = forward.enumerate_visible(pl, q2, x2, g0)
    sel = S["t"] == t
    assert np.array_equal(S["m"][sel], S2["m"]) and np.array_equal(S["n"][sel], S2["n"])
    assert np.allclose(S["s12"][sel], S2["s12"], atol=1e-9)


def test_harmonic_merge():
    pl, g, q, x = _sample(seed=11, n=20, n_rot=6)
    V = forward.enumerate_visible(pl, q, x, g, merge_harmonics=False)
    S = forward.enumerate_visible(pl, q, x, g, merge_harmonics=True)
    assert len(S["m"]) < len(V["m"])
    # every dropped spot coincides with a kept spot of a lower-order parallel plane
    kept = {}
    for k in range(len(S["m"])):
        kept.setdefault((S["n"][k], S["t"][k], S["det"][k]), []).append(k)
    sk = set(zip(S["n"].tolist(), S["t"].tolist(), S["det"].tolist(), S["m"].tolist()))
    for k in range(len(V["m"])):
        key = (V["n"][k], V["t"][k], V["det"][k], V["m"][k])
        if key in sk:
            continue
        cands = kept[key[:3]]
        d = [np.linalg.norm(S["s12"][c] - V["s12"][k]) for c in cands]
        c = cands[int(np.argmin(d))]
        assert min(d) < 1e-9
        assert pl["nsq"][S["m"][c]] < pl["nsq"][V["m"][k]]
        assert np.allclose(np.cross(pl["hkl"][S["m"][c]], pl["hkl"][V["m"][k]]), 0)


def test_eval_fixed_matches_enumerate():
    pl, g, q, x = _sample(seed=13, n=4, n_rot=5)
    S = forward.enumerate_visible(pl, q, x, g)
    ev = forward.eval_fixed(pl, q, x, g, S["m"], S["n"], S["t"], S["det"])
    assert np.allclose(ev["s12"], S["s12"], atol=1e-10)
    assert np.allclose(ev["v"], ev["tau"][:, None] * ev["r"])
    assert np.allclose(ev["s"], ev["y"] + ev["v"])


def test_simulator_counts_and_noise():
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry.from_preset(p)
    q, x = ig.random_grains(p)
    sim = simulate.simulate(pl, q, x, g, p.sigma_mm, p.outlier_frac, p.seed, p.distance)
    sim2 = simulate.simulate(pl, q, x, g, p.sigma_mm, p.outlier_frac, p.seed, p.distance)
    assert np.array_equal(sim["p12"], sim2["p12"])
    n_out = (sim["grain"] < 0).sum()
    assert n_out == np.sum(np.floor(p.outlier_frac * sim["n_true"] + 0.5))
    assert np.all(np.max(np.abs(sim["p12"]), axis=1) < 100.0)
    assert np.all(np.diff(sim["block"]) >= 0)
    # noise-free spots sit exactly on the model spots; noisy ones scatter by ~sigma
    clean = simulate.simulate(pl, q, x, g, 0.0, 0.0, p.seed, p.distance)
    S = forward.enumerate_visible(pl, q, x, g)
    assert len(clean["p12"]) == len(S["m"])
    a = np.sort(np.round(clean["p12"], 9), axis=0)
    b = np.sort(np.round(S["s12"], 9), axis=0)
    assert np.allclose(a, b)


def test_simulator_noise_scale():
    p = ig.MEDIUM
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry(6, np.deg2rad(30.0), p.detectors, p.lam_min, p.lam_max)
    q, x = ig.random_grains(p, n=40)
    sim = simulate.simulate(pl, q, x, g, 0.5, 0.0, 99, p.distance)
    S = forward.enumerate_visible(pl, q, x, g)
    key = {(int(n), int(m), int(b)): k for k, (n, m, b) in enumerate(zip(S["n"], S["m"], S["block"]))}
    d = []
    for i in range(len(sim["p12"])):
        k = key[(int(sim["grain"][i]), int(sim["plane"][i]), int(sim["block"][i]))]
        # angle between noisy and true ray times D ~ sigma per tangent axis
        y = np.einsum("ab,b->a", g.G[S["t"][k]], x[S["n"][k]])
        pl_ = np.r_[S["s"][k][0], sim["p12"][i]]
        rn = (pl_ - y) / np.linalg.norm(pl_ - y)
        d.append(np.linalg.norm(rn - S["r"][k]) * p.distance)
    d = np.array(d)
    # |tangent noise| is Rayleigh with scale sigma: mean sigma sqrt(pi/2)
    assert d.mean() == pytest.approx(0.5 * np.sqrt(np.pi / 2), rel=0.08)
