"""Pins of the oracle's prototype scoring: spot-pair candidates, single-grain
refinement, the SPOT set function (submodularity, greedy guarantee, brute
force) and the number of prototypes."""
import itertools
import math

import numpy as np
import pytest

import inputgen as ig
from oracle import candidates, cost, crystal, forward, metrics, simulate, single


def _noise_free(n_grains=3, n_rot=6, seed=1):
    p = ig.MEDIUM
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry(n_rot, np.deg2rad(30.0), p.detectors, p.lam_min, p.lam_max)
    q, x = ig.random_grains(p, n=n_grains, seed=seed)
    return p, pl, g, q, x


def test_family_representatives():
    pl = crystal.cubic_planes(2.87, "I", 30)
    reps = candidates.family_representatives(pl)
    # every plane is a proper-rotation image of exactly one representative
    G = crystal.cubic_group()
    orbit = {}
    for r in reps:
        for S in G:
            orbit.setdefault(tuple(np.rint(S @ pl["hkl"][r]).astype(int)), set()).add(int(r))
    for h in pl["hkl"].tolist():
        assert len(orbit[tuple(h)]) == 1
    # families with all indices distinct and non-zero ({321}, {431}, ...) split in two
    fams = {tuple(sorted(np.abs(h))) for h in pl["hkl"].tolist()}
    split = sum(1 for f in fams if len(set(f)) == 3 and 0 not in f)
    assert len(reps) == len(fams) + split


def test_spot_normal_inverts_forward_model():
    p, pl, g, q, x = _noise_free()
    x = np.zeros_like(x)
    S = forward.enumerate_visible(pl, q, x, g)
    n, sth, _ = candidates.spot_normals(g, S["s12"], S["block"])
    R = crystal.quat_to_R(q)
    w = np.einsum("jab,jb->ja", R[S["n"]], pl["w"][S["m"]])      # R w: sample-frame normal
    assert np.allclose(n, w, atol=1e-12)
    assert np.allclose(2 * pl["d"][S["m"]] * sth, S["lam"], rtol=1e-12)


def test_same_grain_pair_gives_exact_orientation():
    p, pl, g, q, x = _noise_free(n_grains=2, seed=4)
    x = np.zeros_like(x)
    sim = simulate.simulate(pl, q, x, g, 0.0, 0.0, 9, p.distance)
    c = candidates.generate(pl, g, sim["p12"], sim["offsets"], 200, 3)
    same = sim["grain"][c["a"]] == sim["grain"][c["b"]]
    assert same.any()
    mis = np.degrees(metrics.misorientation(c["q"][:, None, :], q[None, :, :])).min(axis=1)
    # each same-grain pair with its true (hkl) hypothesis reproduces the grain exactly
    good_pairs = set(c["pair"][same & (mis < 1e-7)].tolist())
    same_pairs = set(c["pair"][same].tolist())
    assert len(good_pairs) >= 0.9 * len(same_pairs)


def test_refine_converges_from_nearby_start():
    p, pl, g, q, x = _noise_free(n_grains=4, n_rot=8, seed=6)
    sim = simulate.simulate(pl, q, x, g, 0.5, 0.2, 2, p.distance)
    c_out = cost.c_out(0.5, p.distance)
    q0, x0 = ig.perturb_grains(q[:1], x[:1], 1.0, 0.0, 3)
    qq, xx, mod = single.refine(pl, g, p.distance, sim["p12"], sim["offsets"], q0[0], np.zeros(3), 0.5, c_out)
    assert np.degrees(metrics.misorientation(qq, q[0])) < 0.05
    assert np.linalg.norm(xx - x[0]) < 0.3
    un, nm, rows, vals = single.score(pl, g, p.distance, sim["p12"], sim["offsets"], mod, qq, xx, 0.5, c_out)
    assert un < 0.1 * nm
    assert np.all(vals > -c_out / (2 * 0.25))


def _random_cols(rng, n_rows, n_cand, phi):
    cols = []
    for _ in range(n_cand):
        r = np.sort(rng.choice(n_rows, size=rng.integers(1, n_rows // 2), replace=False))
        cols.append((r, phi + rng.uniform(0.0, 3.0, len(r))))
    return cols


def test_spot_function_properties():
    rng = np.random.default_rng(0)
    phi = -4.5
    for _ in range(5):
        cols = _random_cols(rng, 20, 7, phi)
        f = lambda S: single.spot_value(cols, 20, phi, S)
        assert f([]) == 0.0
        for A in itertools.combinations(range(7), 2):
            B = list(A) + [int(rng.integers(7))]
            for e in range(7):
                # monotone and submodular: gain of e on A >= gain on the superset B
                assert f(list(A) + [e]) >= f(list(A)) - 1e-12
                assert f(list(A) + [e]) - f(list(A)) >= f(B + [e]) - f(B) - 1e-12


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_greedy_guarantee_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    phi = -4.5
    cols = _random_cols(rng, 25, 10, phi)
    k = 3
    picks, gains = single.greedy(cols, 25, phi, k_max=k)
    fg = single.spot_value(cols, 25, phi, picks)
    opt = max(single.spot_value(cols, 25, phi, list(S)) for S in itertools.combinations(range(10), k))
    assert fg >= (1 - 1 / math.e) * opt - 1e-12
    assert np.isclose(np.sum(gains), fg)
    assert np.all(np.diff(gains) <= 1e-12)          # increments never grow (submodularity)


def test_prototype_count_step_one_is_the_largest_drop():
    """With a step of one pick the rule is the printed second difference:
    argmax_k (Delta_k - Delta_{k+1}), Delta beyond the picks 0 (brute force)."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        g = np.sort(rng.uniform(0, 10, rng.integers(1, 40)))[::-1]
        d = np.append(g, 0.0)
        assert single.n_prototypes(g, h=1) == int(np.argmax(d[:-1] - d[1:])) + 1


def test_prototype_count_is_not_decided_by_one_gap():
    """300 true grains whose increments fall by 9 per pick from 3800 (to about
    1060), except one gap of 50 between picks 2 and 3 (the largest single gap,
    as the top order statistics of the grains' gains give), then a sustained
    fall of 20 per pick over 40 picks and a tail falling by 0.4 per pick to
    about 0: the printed step peaks at the one gap (k = 2), the 8-pick
    difference at the fall (k ~ 300)."""
    top = 3800.0 - 9.0 * np.arange(300)
    top[2:] -= 50.0
    fall = top[-1] - 20.0 * np.arange(1, 41)
    tail = fall[-1] - 0.395 * np.arange(1, 651)
    g = np.concatenate([top, fall, tail])
    assert np.all(np.diff(g) < 0)
    assert single.n_prototypes(g, h=1) == 2
    k = single.n_prototypes(g)
    assert 296 <= k <= 312, k


def test_number_of_prototypes_on_separated_grains():
    # 4 disjoint groups of rows, each covered by 3 near-identical candidates
    phi = -4.5
    cols = []
    for gidx in range(4):
        rows = np.arange(gidx * 30, gidx * 30 + 30)
        for d in range(3):
            cols.append((rows, phi + 3.0 - 0.01 * d + 0.001 * np.arange(30)))
    picks, gains = single.greedy(cols, 120, phi)
    assert single.n_prototypes(gains) == 4
    assert sorted(p // 3 for p in picks[:4]) == [0, 1, 2, 3]
