"""Cubic crystallography for the oracle (paper Sec. 3.1 and Sec. 3.3).

Test infrastructure: FP64, plain NumPy.

The paper takes the Miller-plane set {(w_m, d_m)} as an input (Sec. 3.3).  It
does not say how to build it; the reading used here: every signed integer
triple (h,k,l) != 0 with N = h^2+k^2+l^2 <= n_max that survives the lattice's
extinction rule (body-centred: h+k+l even; face-centred: h,k,l all even or all
odd; primitive: none), with unit normal w = (h,k,l)/sqrt(N) and spacing
d = a/sqrt(N) (Sec. 3.1), ordered by (N, h, k, l).

Parallel planes [h,k,l] and [nh,nk,nl] diffract along the same ray.  For each
plane, ``harmonic_prev`` is the index of the allowed plane in the same
direction with the next smaller N (or -1).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def allowed(h, k, l, centering):
    if centering == "P":
        return True
    if centering == "I":
        return (h + k + l) % 2 == 0
    if centering == "F":
        par = {h % 2, k % 2, l % 2}
        return len(par) == 1
    raise ValueError(centering)


def cubic_planes(a, centering, n_max):
    """Plane list: dict with hkl [M,3] int, w [M,3], d [M], nsq [M], harmonic_prev [M]."""
    lim = int(math.isqrt(n_max))
    rows = []
    for h in range(-lim, lim + 1):
        for k in range(-lim, lim + 1):
            for l in range(-lim, lim + 1):
                n = h * h + k * k + l * l
                if n == 0 or n > n_max or not allowed(h, k, l, centering):
                    continue
                rows.append((n, h, k, l))
    rows.sort()
    hkl = np.array([[r[1], r[2], r[3]] for r in rows], dtype=np.int64)
    nsq = np.array([r[0] for r in rows], dtype=np.int64)
    w = hkl / np.sqrt(nsq)[:, None]
    d = a / np.sqrt(nsq)
    index = {tuple(v): i for i, v in enumerate(hkl.tolist())}
    prev = np.full(len(rows), -1, dtype=np.int64)
    for i, (h, k, l) in enumerate(hkl.tolist()):
        g = math.gcd(math.gcd(abs(h), abs(k)), abs(l))
        base = (h // g, k // g, l // g)
        # allowed parallel planes with a smaller multiple, largest multiple first
        for mult in range(g - 1, 0, -1):
            key = (base[0] * mult, base[1] * mult, base[2] * mult)
            if key in index:
                prev[i] = index[key]
                break
    return {"hkl": hkl, "w": w, "d": d, "nsq": nsq, "harmonic_prev": prev}


def quat_to_R(q):
    """Rotation matrices [n,3,3] of unit quaternions (w,x,y,z) [n,4]."""
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def R_to_quat(R):
    """Unit quaternion (w >= 0) of a single rotation matrix (Shepperd's method)."""
    R = np.asarray(R, dtype=np.float64)
    tr = np.trace(R)
    cand = np.array([tr, R[0, 0], R[1, 1], R[2, 2]])
    i = int(np.argmax(cand))
    if i == 0:
        w = math.sqrt(1.0 + tr) / 2.0
        q = [w, (R[2, 1] - R[1, 2]) / (4 * w), (R[0, 2] - R[2, 0]) / (4 * w),
             (R[1, 0] - R[0, 1]) / (4 * w)]
    elif i == 1:
        x = math.sqrt(1.0 + 2 * R[0, 0] - tr) / 2.0
        q = [(R[2, 1] - R[1, 2]) / (4 * x), x, (R[0, 1] + R[1, 0]) / (4 * x),
             (R[0, 2] + R[2, 0]) / (4 * x)]
    elif i == 2:
        y = math.sqrt(1.0 + 2 * R[1, 1] - tr) / 2.0
        q = [(R[0, 2] - R[2, 0]) / (4 * y), (R[0, 1] + R[1, 0]) / (4 * y), y,
             (R[1, 2] + R[2, 1]) / (4 * y)]
    else:
        z = math.sqrt(1.0 + 2 * R[2, 2] - tr) / 2.0
        q = [(R[1, 0] - R[0, 1]) / (4 * z), (R[0, 2] + R[2, 0]) / (4 * z),
             (R[1, 2] + R[2, 1]) / (4 * z), z]
    q = np.array(q)
    q /= np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def rot_z(omega):
    """Sample rotation Gamma_t about the (0,0,1) axis (Sec. 3.3) [..,3,3]."""
    c, s = np.cos(omega), np.sin(omega)
    G = np.zeros(np.shape(omega) + (3, 3))
    G[..., 0, 0] = c
    G[..., 0, 1] = -s
    G[..., 1, 0] = s
    G[..., 1, 1] = c
    G[..., 2, 2] = 1.0
    return G


def scan_rotations(n_rot, domega_rad, omega0=0.0):
    return rot_z(omega0 + domega_rad * np.arange(n_rot))


def rodrigues(omega):
    """exp([omega]_x) for one axis-angle vector."""
    omega = np.asarray(omega, dtype=np.float64)
    th = np.linalg.norm(omega)
    K = np.array([[0, -omega[2], omega[1]], [omega[2], 0, -omega[0]], [-omega[1], omega[0], 0]])
    if th < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K


def cubic_group():
    """The 24 proper rotations of the cube: signed permutation matrices, det +1."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3))
            for r, c in enumerate(perm):
                M[r, c] = signs[r]
            if np.linalg.det(M) > 0:
                out.append(M)
    return np.array(out)
