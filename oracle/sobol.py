"""Sobol-grid starts of single-grain fitting (paper Sec. 6.1): a Sobol
sequence over the six-dimensional (R, x) space, orientations as modified
Rodrigues parameters (MRP) restricted to the cubic fundamental zone,
positions within the sample's bounds.

Test infrastructure: FP64 and exact integers, plain Python / NumPy.

Sobol points (Sobol 1967; Bratley and Fox 1988): coordinate d of point n is
the XOR of the direction numbers V_d[k] over the bits k set in the Gray code
n ^ (n >> 1), divided by 2^32 (the Antonov-Saleev order, point 0 = origin).
Dimension 1 has V[k] = 2^(31-k); dimensions 2..6 take the primitive
polynomials and initial numbers m_1..m_s of Joe and Kuo's table (2008, file
new-joe-kuo-6.21201), extended by the recurrence
  V[k] = V[k-s] ^ (V[k-s] >> s) ^ XOR_{i=1..s-1, a_i = 1} V[k-i].
Readings:
  * MRP: p = n tan(theta/4) for the rotation by theta about n; the unit
    quaternion is ((1 - |p|^2), 2 p) / (1 + |p|^2);
  * the orientation grid is the MRP cube |p_i| <= tan(pi/16) (the largest MRP
    component of the cubic fundamental zone, a 45-degree rotation about a
    cube axis), u in [0,1) mapped to (2u - 1) tan(pi/16); a point is kept when
    its rotation lies in the cubic (432) fundamental zone: Rodrigues vector
    r = (q1, q2, q3) / q0 with |r_i| <= tan(pi/8) for every i and
    |r_1| + |r_2| + |r_3| <= 1;
  * positions: (2u - 1) times the caller's half extents of the sample box;
  * points keep their Sobol index order.
"""
from __future__ import annotations

import math

import numpy as np

BITS = 32
# (degree s, coefficients a, initial m_1..m_s) of dimensions 2..6
JOE_KUO = [(1, 0, [1]), (2, 1, [1, 3]), (3, 1, [1, 3, 1]), (3, 2, [1, 1, 1]), (4, 1, [1, 1, 3, 3])]
MRP_HALF = math.tan(math.pi / 16)
R_FACE = math.tan(math.pi / 8)


def directions():
    """Direction numbers [6][32] (integers; V[d][k] for bit k = 0..31)."""
    out = [[1 << (BITS - 1 - k) for k in range(BITS)]]
    for s, a, m in JOE_KUO:
        V = [0] * (BITS + 1)
        for k in range(1, s + 1):
            V[k] = m[k - 1] << (BITS - k)
        for k in range(s + 1, BITS + 1):
            v = V[k - s] ^ (V[k - s] >> s)
            for i in range(1, s):
                if (a >> (s - 1 - i)) & 1:
                    v ^= V[k - i]
            V[k] = v
        out.append(V[1:])
    return out


def points(first, n, dims=6):
    """Sobol points first .. first+n-1 in [0, 1)^dims."""
    V = directions()
    out = np.zeros((n, dims))
    for r in range(n):
        idx = first + r
        g = idx ^ (idx >> 1)
        for d in range(dims):
            x = 0
            k = 0
            while g >> k:
                if (g >> k) & 1:
                    x ^= V[d][k]
                k += 1
            out[r, d] = x / 2.0 ** BITS
    return out


def mrp_to_quat(p):
    p = np.asarray(p, dtype=np.float64)
    s = np.sum(p * p, axis=-1, keepdims=True)
    return np.concatenate([1.0 - s, 2.0 * p], axis=-1) / (1.0 + s)


def in_cubic_fz(q):
    """Whether each rotation (unit quaternion, any sign) lies in the cubic
    fundamental zone (Rodrigues-vector test)."""
    q = np.asarray(q, dtype=np.float64)
    q = np.where(q[..., :1] < 0, -q, q)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = q[..., 1:] / q[..., :1]
    a = np.abs(r)
    return np.all(a <= R_FACE, axis=-1) & (np.sum(a, axis=-1) <= 1.0)


def starts(first, n, x_half, mrp_half=MRP_HALF, restrict_fz=True):
    """Starts from Sobol points first .. first+n-1: (kept indices, q [k,4]
    with q0 >= 0, x [k,3])."""
    u = points(first, n)
    p = (2.0 * u[:, :3] - 1.0) * mrp_half
    q = mrp_to_quat(p)
    x = (2.0 * u[:, 3:] - 1.0) * np.asarray(x_half, dtype=np.float64)
    keep = in_cubic_fz(q) if restrict_fz else np.ones(n, bool)
    idx = np.flatnonzero(keep)
    return first + idx, q[idx], x[idx]
