"""The zero radius of the refinement passes' cell index, checked in FP64 on
random detector geometry: beyond R (the radius the library computes from
t0 = sqrt(2 T |v|^2 / v_n^2), R = t0 |v| / (1 - t0)), every in-plane offset
delta gives a chord cost c' = 1 - cos(v, v + delta) with K c' >= T."""
import numpy as np


def _chord(v, d):
    """1 - cos of the angle between v and v + d (FP64)."""
    w = v + d
    return 1.0 - np.sum(v * w, axis=-1) / (np.linalg.norm(v, axis=-1) * np.linalg.norm(w, axis=-1))


def test_beyond_the_zero_radius_every_term_underflows():
    rng = np.random.default_rng(7)
    T = 160.0
    n_checked = 0
    for _ in range(200):
        # a detector plane (unit normal nu) and a ray vector v towards it
        nu = rng.standard_normal(3)
        nu /= np.linalg.norm(nu)
        a = np.cross(nu, rng.standard_normal(3))
        a /= np.linalg.norm(a)
        b = np.cross(nu, a)
        vn = rng.uniform(0.1, 1.0)
        par = np.sqrt(1.0 - vn ** 2)
        ang = rng.uniform(0, 2 * np.pi)
        v = rng.uniform(100.0, 400.0) * (vn * nu + par * (np.cos(ang) * a + np.sin(ang) * b))
        vv = v @ v
        for eps_scale in (0.5, 3.0, 30.0, 300.0):
            K = 2.0 * 150.0 ** 2 / (eps_scale * 1.0) * 1.4426950408889634
            t2 = 2.0 * (T / K) * vv / (v @ nu) ** 2
            if not ((v @ nu) ** 2 >= 1e-4 * vv and t2 < 0.81):
                continue
            t0 = np.sqrt(t2)
            R = t0 * np.sqrt(vv) / (1.0 - t0)
            # offsets in the plane at R and beyond, every direction
            phi = rng.uniform(0, 2 * np.pi, 512)
            r = R * (1.0 + rng.exponential(0.5, 512) * (rng.random(512) < 0.5))
            d = r[:, None] * (np.cos(phi)[:, None] * a + np.sin(phi)[:, None] * b)
            assert np.all(K * _chord(v, d) >= T * (1.0 - 1e-9))
            n_checked += 1
    assert n_checked > 300
