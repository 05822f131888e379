"""Pins of the Sobol-grid starts: the points against SciPy's unscrambled
Sobol generator (Joe-Kuo direction numbers), the MRP map against the
rotation it must give, and the fundamental-zone test against brute force
over the 24 cube rotations."""
import math

import numpy as np
import pytest
from scipy.stats import qmc

import inputgen as ig
from oracle import crystal, sobol


def test_points_match_scipy():
    ref = qmc.Sobol(d=6, scramble=False).random(4096)
    assert np.array_equal(sobol.points(0, 4096), ref)
    # any window of the sequence
    assert np.array_equal(sobol.points(1000, 37), ref[1000:1037])


def test_mrp_is_a_quarter_angle_tangent():
    rng = np.random.default_rng(1)
    for _ in range(20):
        axis = rng.standard_normal(3)
        axis /= np.linalg.norm(axis)
        th = rng.uniform(0.0, math.pi)
        q = sobol.mrp_to_quat(axis * math.tan(th / 4))
        R = crystal.quat_to_R(q)
        # rotation by th about axis (Rodrigues' formula)
        K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
        Rt = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K
        assert np.allclose(R, Rt, atol=1e-12)
        assert np.linalg.norm(q) == pytest.approx(1.0)


def _angle(R):
    return math.acos(max(-1.0, min(1.0, (np.trace(R) - 1) / 2)))


def test_fundamental_zone_is_the_smallest_angle_representative():
    """A rotation lies in the cubic fundamental zone exactly when no cube
    rotation S gives R S a smaller rotation angle (away from the boundary)."""
    rng = np.random.default_rng(2)
    S = crystal.cubic_group()
    assert len(S) == 24
    q = ig.random_quaternions(rng, 3000)
    inside = sobol.in_cubic_fz(q)
    Rs = crystal.quat_to_R(q)
    n_checked = 0
    for R, ins in zip(Rs, inside):
        a = np.array([_angle(R @ s) for s in S])
        own = _angle(R)
        others = np.sort(a)
        if abs(own - others[0]) < 1e-9 and others[1] - others[0] < 1e-6:
            continue          # on the boundary: two representatives tie
        assert ins == (own <= others[0] + 1e-12)
        n_checked += 1
    assert n_checked > 2900
    # every orientation has exactly one representative inside (almost surely)
    for R in Rs[:200]:
        reps = [crystal.R_to_quat(R @ s) for s in S]
        assert int(np.sum(sobol.in_cubic_fz(np.array(reps)))) == 1
    # the zone holds 1/24 of the rotations
    assert np.mean(inside) == pytest.approx(1 / 24, abs=0.012)


def test_mrp_cube_contains_the_zone():
    """Every rotation of the zone has MRP components within tan(pi/16)."""
    rng = np.random.default_rng(3)
    q = ig.random_quaternions(rng, 20000)
    q = q[sobol.in_cubic_fz(q)]
    q = np.where(q[:, :1] < 0, -q, q)
    p = q[:, 1:] / (1 + q[:, :1])
    assert np.max(np.abs(p)) <= sobol.MRP_HALF + 1e-12
    assert np.max(np.abs(p)) > 0.9 * sobol.MRP_HALF


def test_starts():
    idx, q, x = sobol.starts(5, 2000, (2.5, 2.5, 2.5))
    assert np.all(np.diff(idx) > 0) and idx[0] >= 5
    assert np.all(sobol.in_cubic_fz(q)) and np.all(q[:, 0] > 0)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0)
    assert np.all(np.abs(x) <= 2.5)
    # the kept fraction is the zone's share of the MRP cube (Monte Carlo estimate)
    rng = np.random.default_rng(4)
    pr = rng.uniform(-sobol.MRP_HALF, sobol.MRP_HALF, (200000, 3))
    share = np.mean(sobol.in_cubic_fz(sobol.mrp_to_quat(pr)))
    assert len(idx) / 2000 == pytest.approx(share, abs=0.01)
    idx2, q2, x2 = sobol.starts(5, 2000, (2.5, 2.5, 2.5), restrict_fz=False)
    assert len(idx2) == 2000
