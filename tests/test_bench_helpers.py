"""The bench's recall and misorientation (host code that turns indexing
results into the time-to-index figures), checked against the oracle's
rotation-matrix misorientation and by construction."""
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from oracle import crystal, metrics  # noqa: E402


def _unit(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _turn(q, angle_deg, rng):
    """Each quaternion turned by angle_deg about a random axis."""
    ax = rng.standard_normal((len(q), 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    h = math.radians(angle_deg) / 2
    d = np.concatenate([np.full((len(q), 1), math.cos(h)), math.sin(h) * ax], axis=1)
    w1, x1, y1, z1 = d.T
    w2, x2, y2, z2 = q.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=1)


def test_misorientation_matches_oracle_over_the_cubic_group():
    rng = np.random.default_rng(1)
    qa, qb = _unit(rng, 40), _unit(rng, 30)
    got = bench.misorientation_deg(qa, qb)
    ref = np.degrees(metrics.misorientation(qa[:, None, :], qb[None, :, :]))
    assert np.max(np.abs(got - ref)) < 1e-6
    assert got.max() <= 62.8 + 1e-6          # the cubic group's largest disorientation


def test_misorientation_ignores_cubic_symmetry_and_sign():
    rng = np.random.default_rng(2)
    q = _unit(rng, 10)
    R = crystal.quat_to_R(q)
    group = crystal.cubic_group()
    assert len(group) == 24
    for S in group:
        qs = np.array([crystal.R_to_quat(R[k] @ S) for k in range(len(q))])
        assert np.max(np.diag(bench.misorientation_deg(q, qs))) < 1e-5
    assert np.max(np.diag(bench.misorientation_deg(q, -q))) < 1e-5   # acos near 1: ~1e-6 deg rounding
    turned = _turn(q, 0.3, rng)
    assert np.allclose(np.diag(bench.misorientation_deg(q, turned)), 0.3, atol=1e-6)


def test_recall_is_one_to_one_within_both_bounds():
    rng = np.random.default_rng(3)
    q = _unit(rng, 20)
    x = rng.uniform(-2, 2, (20, 3))
    est_q = _turn(q, 0.1, rng)
    est_x = x + 0.1
    perm = rng.permutation(20)
    assert bench.recall(est_q[perm], est_x[perm], q, x) == 20
    # a duplicate estimate matches no second grain
    assert bench.recall(np.concatenate([est_q, est_q[:3]]), np.concatenate([est_x, est_x[:3]]), q, x) == 20
    # one estimate off in position, one off in orientation
    est_x[4] += np.array([0.6, 0.0, 0.0])
    est_q[7] = _turn(q[7:8], 0.3, rng)[0]
    assert bench.recall(est_q, est_x, q, x) == 18
    assert bench.recall(np.zeros((0, 4)), np.zeros((0, 3)), q, x) == 0


def test_geometric_schedule_endpoints():
    s = bench._geometric(7.9, 1.11, 20)
    assert len(s) == 20 and abs(s[0] - 7.9) < 1e-12 and abs(s[-1] - 1.11) < 1e-12
    r = np.array(s[1:]) / np.array(s[:-1])
    assert np.allclose(r, r[0])
    assert bench._geometric(3.0, 1.0, 1) == [3.0]
