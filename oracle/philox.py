"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11), written from its published
definition, plus the uniform and Gaussian maps the simulator uses.

Test infrastructure (oracle side).  The HIP library implements the same
published generator independently.

Round function on counter (c0,c1,c2,c3) with key (k0,k1):
  (hi0, lo0) = mulhilo32(0xD2511F53, c0); (hi1, lo1) = mulhilo32(0xCD9E8D57, c2)
  c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
ten rounds, the key bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85)
between rounds.

Counter layout used by the simulator (stream id in the last word):
  ray noise of spot (grain n, rotation t, plane m, detector d):
      (n, t, m + 65536 d, 1)
  position of outlier k in block (t, d):  (k, t, 65536 d, 2)
  order key of true spot (n,t,m,d):       (n, t, m + 65536 d, 3)
  order key of outlier k in block (t,d):  (k, t, 65536 d, 4)
Key = (seed & 0xffffffff, seed >> 32).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)

STREAM_NOISE = 1
STREAM_OUTLIER = 2
STREAM_KEY_TRUE = 3
STREAM_KEY_OUT = 4


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Inputs: uint32-valued integer arrays (broadcast).
    Returns four uint64 arrays holding the uint32 outputs."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for r in range(10):
        p0 = M0 * c0           # < 2^64: exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> S32, p0 & MASK
        hi1, lo1 = p1 >> S32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        if r < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def seed_key(seed):
    seed = int(seed)
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def uniform01(x):
    """uint32 -> (0,1): (x + 0.5) / 2^32, exact in FP64."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


def box_muller(u1, u2):
    """Two independent standard normals from two uniforms on (0,1)."""
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def normals3(c0, c1, c2, c3, seed):
    """Three standard normals per counter (words 0,1 -> z0,z1; words 2,3 -> z2)."""
    k0, k1 = seed_key(seed)
    x0, x1, x2, x3 = philox4x32_10(c0, c1, c2, c3, k0, k1)
    z0, z1 = box_muller(uniform01(x0), uniform01(x1))
    z2, _ = box_muller(uniform01(x2), uniform01(x3))
    return np.stack([z0, z1, z2], axis=-1)


def uniforms2(c0, c1, c2, c3, seed):
    k0, k1 = seed_key(seed)
    x0, x1, _, _ = philox4x32_10(c0, c1, c2, c3, k0, k1)
    return uniform01(x0), uniform01(x1)


def key64(c0, c1, c2, c3, seed):
    """64-bit order key: (word0 << 32) | word1."""
    k0, k1 = seed_key(seed)
    x0, x1, _, _ = philox4x32_10(c0, c1, c2, c3, k0, k1)
    return (x0 << S32) | x1
