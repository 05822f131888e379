"""Pins of the oracle's plane lists, rotations and random numbers."""
import itertools

import numpy as np
import pytest

from oracle import crystal, philox


@pytest.mark.parametrize("a,cen,nmax,count", [(2.87, "I", 14, 134), (2.87, "I", 30, 368),
                                              (3.52, "F", 40, 282), (3.52, "F", 30, 168),
                                              (3.0, "P", 3, 26)])
def test_plane_counts(a, cen, nmax, count):
    # counts follow from enumerating the extinction rules by hand; P with N<=3 is
    # the 6 {100} + 12 {110} + 8 {111} planes
    pl = crystal.cubic_planes(a, cen, nmax)
    assert len(pl["hkl"]) == count


def test_plane_spacing_and_normals():
    pl = crystal.cubic_planes(2.87, "I", 30)
    n = pl["nsq"]
    assert np.allclose(pl["d"], 2.87 / np.sqrt(n))
    assert np.allclose(np.linalg.norm(pl["w"], axis=1), 1.0)
    assert np.all((pl["hkl"].sum(axis=1) % 2) == 0)
    assert np.all(np.diff(n) >= 0)


@pytest.mark.parametrize("cen,nmax", [("I", 30), ("F", 40)])
def test_plane_list_closed_under_cubic_group(cen, nmax):
    pl = crystal.cubic_planes(3.0, cen, nmax)
    s = {tuple(v) for v in pl["hkl"].tolist()}
    for S in crystal.cubic_group():
        for v in pl["hkl"]:
            assert tuple(int(x) for x in S @ v) in s
    for v in pl["hkl"].tolist():
        assert tuple(-x for x in v) in s


def test_harmonic_prev_chain():
    pl = crystal.cubic_planes(2.87, "I", 30)
    idx = {tuple(v): i for i, v in enumerate(pl["hkl"].tolist())}
    prev = pl["harmonic_prev"]
    assert prev[idx[(2, 2, 0)]] == idx[(1, 1, 0)]
    assert prev[idx[(3, 3, 0)]] == idx[(2, 2, 0)]
    assert prev[idx[(4, 0, 0)]] == idx[(2, 0, 0)]
    assert prev[idx[(2, 0, 0)]] == -1            # (1,0,0) is extinct in BCC
    assert prev[idx[(4, 2, 2)]] == idx[(2, 1, 1)]
    assert prev[idx[(3, 1, 0)]] == -1
    for i, p in enumerate(prev):
        if p >= 0:
            a, b = pl["hkl"][i], pl["hkl"][p]
            assert np.allclose(np.cross(a, b), 0) and a @ b > 0 and pl["nsq"][p] < pl["nsq"][i]


def test_cubic_group():
    G = crystal.cubic_group()
    assert len(G) == 24
    keys = {tuple(np.rint(M).astype(int).ravel()) for M in G}
    for A, B in itertools.product(G, G):
        assert tuple(np.rint(A @ B).astype(int).ravel()) in keys


def test_quaternion_rotation_roundtrip():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((50, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    R = crystal.quat_to_R(q)
    assert np.allclose(np.einsum("nab,nac->nbc", R, R), np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(R), 1.0)
    for qq, RR in zip(q, R):
        assert np.allclose(crystal.R_to_quat(RR), qq, atol=1e-12)
    # 90 degrees about z maps x to y
    qz = np.array([np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)])
    assert np.allclose(crystal.quat_to_R(qz) @ [1, 0, 0], [0, 1, 0])
    assert np.allclose(crystal.rot_z(np.pi / 2) @ [1, 0, 0], [0, 1, 0])


def test_rodrigues_matches_quaternion():
    w = np.array([0.3, -0.2, 0.5])
    th = np.linalg.norm(w)
    q = np.concatenate([[np.cos(th / 2)], np.sin(th / 2) * w / th])
    assert np.allclose(crystal.rodrigues(w), crystal.quat_to_R(q), atol=1e-14)


def test_philox_known_answers():
    # known-answer vectors published with the Random123 reference implementation
    cases = [((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
             ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
             ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
              (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for c, k, want in cases:
        got = philox.philox4x32_10(*c, *k)
        assert tuple(int(v) for v in got) == want


def test_philox_normals_statistics():
    i = np.arange(200000)
    z = philox.normals3(i, 7, 3, philox.STREAM_NOISE, 12345)
    assert abs(z.mean()) < 0.01
    assert abs(z.std() - 1.0) < 0.01
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.01
