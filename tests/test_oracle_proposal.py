"""Pins of the oracle's learned-proposal inputs: cheap-support features,
training labels and top-fraction selection."""
import numpy as np

import inputgen as ig
from oracle import crystal, forward, proposal, simulate


def _setup(n_grains=3, n_rot=12, seed=2):
    p = ig.MEDIUM
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry(n_rot, np.deg2rad(180.0 / n_rot), p.detectors, p.lam_min, p.lam_max)
    q, _ = ig.random_grains(p, n=n_grains, seed=seed)
    return p, pl, g, q


def test_probe_rotations_and_planes():
    assert proposal.probe_rotations(0, 60) == [20, 40]
    assert proposal.probe_rotations(50, 60) == [10, 30]
    assert proposal.probe_rotations(3, 12) == [7, 11]
    pl = crystal.cubic_planes(2.87, "I", 30)
    m = proposal.probe_planes(pl, 134)
    assert np.all(pl["harmonic_prev"][m] < 0) and np.all(m < 134)
    # {200} is the second harmonic of nothing in BCC (100 is extinct), {220} of {110}
    nsq = pl["nsq"][m]
    assert 2 in nsq and 4 in nsq and 8 not in nsq


def test_prediction_matches_vectorised_forward_model():
    p, pl, g, q = _setup()
    mset = proposal.probe_planes(pl, 200)
    sub = {k: v[mset] for k, v in pl.items()}
    sub["harmonic_prev"] = -np.ones(len(mset), dtype=np.int64)
    V = forward.enumerate_visible(sub, q, np.zeros((len(q), 3)), g, merge_harmonics=False)
    for n in range(len(q)):
        R = crystal.quat_to_R(q[n])
        for t in (0, 5, 11):
            got = proposal.predict(pl, g, R, t, mset)
            sel = (V["n"] == n) & (V["t"] == t)
            want = sorted(zip(V["det"][sel].tolist(), V["s12"][sel].tolist()))
            have = sorted((d, s.tolist()) for d, s, _ in got)
            assert len(have) == len(want)
            for (d1, s1), (d2, s2) in zip(have, want):
                assert d1 == d2 and np.allclose(s1, s2, atol=1e-9)


def test_true_orientation_has_full_support():
    p, pl, g, q = _setup()
    x = np.zeros((len(q), 3))
    sim = simulate.simulate(pl, q, x, g, 0.0, 0.0, 5, p.distance)
    # each true grain, also presented in a symmetry-equivalent setting
    S = crystal.cubic_group()[7]
    qs = np.array([crystal.R_to_quat(crystal.quat_to_R(qq) @ S) for qq in q])
    for qq in (q, qs):
        frac, border = proposal.support(pl, g, sim["p12"], sim["offsets"], qq, np.array([0, 3, 8]), 1.0,
                                        len(pl["d"]))
        assert np.all(frac == 1.0)
        assert np.all(border == 0)


def test_support_counts_hits_within_radius():
    p, pl, g, q = _setup(n_grains=1)
    R = crystal.quat_to_R(q[0])
    n_all = len(pl["d"])
    mset = proposal.probe_planes(pl, n_all)
    t0 = next(t for t in range(g.n_rot)
              if len(proposal.predict(pl, g, R, proposal.probe_rotations(t, g.n_rot)[0], mset)) >= 4)
    t1, t2 = proposal.probe_rotations(t0, g.n_rot)
    pred = proposal.predict(pl, g, R, t1, mset)
    # plant a spot 0.9 mm away from the first two predictions, 1.1 mm from the next two
    pts, blocks = [], []
    for i, (d, s12, _) in enumerate(pred[:4]):
        off = 0.9 if i < 2 else 1.1
        pts.append(s12 + np.array([off * 0.6, off * 0.8]))
        blocks.append(t1 * g.n_det + d)
    order = np.argsort(blocks, kind="stable")
    p12 = np.array(pts)[order]
    offsets = forward.block_offsets(np.array(blocks)[order], g.n_blocks)
    frac, _ = proposal.support(pl, g, p12, offsets, q, np.array([t0]), 1.0, n_all)
    assert frac[0, 0] == 2.0 / len(pred)
    assert frac[0, 1] == 0.0


def test_labels():
    q_true = np.array([[1.0, 0, 0, 0], [np.cos(0.3), np.sin(0.3), 0, 0]])
    grain = np.array([0, 0, 1, -1, 1])
    S = crystal.cubic_group()[13]
    q_sym = crystal.R_to_quat(crystal.quat_to_R(q_true[1]) @ S)
    h = np.radians(1.9) / 2
    q_near = np.array([np.cos(h), 0, 0, np.sin(h)])
    h = np.radians(2.1) / 2
    q_far = np.array([np.cos(h), 0, np.sin(h), 0])
    q = np.array([q_near, q_far, q_sym, q_true[1], q_true[0]])
    a = np.array([0, 0, 2, 2, 0])
    b = np.array([1, 1, 4, 3, 2])
    lab, mis = proposal.labels(q, a, b, grain, q_true)
    assert lab.tolist() == [1.0, 0.0, 1.0, 0.0, 0.0]
    assert abs(mis[0] - 1.9) < 1e-9 and abs(mis[1] - 2.1) < 1e-9 and mis[2] < 1e-6
    assert np.isinf(mis[3]) and np.isinf(mis[4])


def test_labels_nearest():
    """By construction: a candidate 0.9 deg from grain 1 (through a cube
    symmetry of it) and 3 deg from grain 0 labels 1 with grain 1; one 1.1 deg
    from grain 0 labels 0 at 1 deg; equal distances go to the lower index."""
    q_true = np.array([[1.0, 0, 0, 0], [np.cos(np.radians(30) / 2), 0, 0, np.sin(np.radians(30) / 2)]])
    S = crystal.cubic_group()[7]
    R1 = crystal.quat_to_R(q_true[1])
    h = np.radians(0.9) / 2
    dR = crystal.quat_to_R(np.array([np.cos(h), np.sin(h), 0, 0]))
    q_a = crystal.R_to_quat(R1 @ dR @ S)
    h = np.radians(1.1) / 2
    q_b = np.array([np.cos(h), 0, np.sin(h), 0])
    h = np.radians(15) / 2
    q_mid = np.array([np.cos(h), 0, 0, np.sin(h)])       # 15 deg from both grains
    lab, mis, near = proposal.labels_nearest(np.array([q_a, q_b, q_mid]), q_true, 1.0)
    assert lab.tolist() == [1.0, 0.0, 0.0]
    assert near.tolist() == [1, 0, 0]
    assert abs(mis[0] - 0.9) < 1e-9 and abs(mis[1] - 1.1) < 1e-9 and abs(mis[2] - 15.0) < 1e-9
    lab, mis, near = proposal.labels_nearest(np.array([q_a]), np.zeros((0, 4)), 1.0)
    assert lab.tolist() == [0.0] and near.tolist() == [-1] and np.isinf(mis[0])


def test_select_top():
    s = np.array([0.5, 0.9, 0.5, 0.9, 0.1])
    assert proposal.select_top(s, 0.6).tolist() == [0, 1, 3]
    assert proposal.select_top(s, 0.5).tolist() == [0, 1, 3]      # ceil(2.5) = 3
    assert proposal.select_top(s, 0.2).tolist() == [1]
    assert proposal.select_top(s, 1.0).tolist() == [0, 1, 2, 3, 4]
    assert proposal.select_top(s, 0.0).tolist() == []
    rng = np.random.default_rng(0)
    v = rng.standard_normal(1000)
    got = proposal.select_top(v, 0.05)
    assert got.tolist() == sorted(np.argsort(-v)[:50].tolist())


def test_same_grain_pairs():
    rng = np.random.default_rng(4)
    n_rot, n_det = 5, 2
    counts = rng.integers(0, 12, n_rot * n_det)
    counts[3] = 0
    offsets = np.concatenate([[0], np.cumsum(counts)])
    grain = rng.integers(-1, 4, offsets[-1])
    a, b = proposal.same_grain_pairs(offsets, grain, n_det, 4000, 123)
    ok = a >= 0
    assert ok.mean() > 0.3
    rot = lambda i: (np.searchsorted(offsets, i, side="right") - 1) // n_det
    assert np.all(b[ok] != a[ok])
    assert np.all(grain[a[ok]] == grain[b[ok]]) and np.all(grain[a[ok]] >= 0)
    assert np.all(rot(a[ok]) == rot(b[ok]))
    # a pair is missing only when a has no mate: outlier, or alone in its rotation
    x0 = __import__("oracle.philox", fromlist=["x"]).philox4x32_10(
        np.arange(4000), 0, 0, proposal.STREAM_SAME_PAIR, 123, 0)[0]
    a_all = (x0 % np.uint64(offsets[-1])).astype(np.int64)
    assert np.array_equal(a[ok], a_all[ok])
    for j in np.nonzero(~ok)[0][:200]:
        i = a_all[j]
        mates = [m for m in range(offsets[-1]) if m != i and rot(m) == rot(i) and grain[m] == grain[i]]
        assert grain[i] < 0 or not mates
    # b is uniform over the mates: for a spot with 3+ mates every mate is drawn
    seen = {}
    for x, y in zip(a[ok], b[ok]):
        seen.setdefault(int(x), set()).add(int(y))
    full = [x for x, ys in seen.items()
            if len(ys) == sum(1 for m in range(offsets[-1]) if m != x and rot(m) == rot(x) and grain[m] == grain[x])]
    assert len(full) > 10
