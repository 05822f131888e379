"""Synthetic detected spots for the oracle (paper Sec. 3.3.1 and Sec. 7 set-up).

Test infrastructure: FP64, plain NumPy.

Detected spots follow the paper's ray-noise model: the true ray r of a model
spot is replaced by a noisy unit ray drawn as an isotropic 3-D Gaussian around
r with standard deviation sigma (angular), normalised (Sec. 3.3.1), and
re-intersected with the detector (Eq. spot_noisy).  The angular sigma is the
detector-plane sigma in mm divided by the detector distance (the paper's
0.4 mm <-> 0.143 deg at 160 mm).  Spots whose noisy ray leaves the detector
are dropped.  Outliers: per (rotation, detector) block, round(f * n_true)
spots uniform over the detector square (Sec. 7: "% of the Laue spot count").
Spots are ordered within each block by a random 64-bit key.

Random numbers come from Philox4x32-10 with the counter layout documented in
oracle/philox.py, so that an independent implementation reproduces them.
"""
from __future__ import annotations

import numpy as np

from . import forward, philox


def simulate(planes, q, x, geom, sigma_mm, outlier_frac, seed, distance):
    """Detected spots of grains (q, x).

    Returns dict: p12 [I,2] (detector-local mm, FP64), block [I], offsets
    [n_blocks+1], grain [I] (-1 for outliers), plane [I] (-1 for outliers),
    n_true per block."""
    vis = forward.enumerate_visible(planes, q, x, geom, merge_harmonics=True)
    sig = sigma_mm / distance
    n, t, m, d = vis["n"], vis["t"], vis["m"], vis["det"]
    c2 = m + 65536 * d
    g = philox.normals3(n, t, c2, philox.STREAM_NOISE, seed)
    rn = vis["r"] + sig * g
    rn /= np.linalg.norm(rn, axis=1, keepdims=True)
    y = np.einsum("jab,jb->ja", geom.G[t], np.atleast_2d(x)[n])
    nu = geom.det_normal[d]
    gam = geom.det_center[d]
    tau = np.einsum("jk,jk->j", gam - y, nu) / np.einsum("jk,jk->j", rn, nu)
    s = y + tau[:, None] * rn
    rel = s - gam
    s12 = np.stack([np.einsum("jk,jk->j", rel, geom.det_a1[d]),
                    np.einsum("jk,jk->j", rel, geom.det_a2[d])], axis=1)
    keep = (tau > 0) & (np.max(np.abs(s12), axis=1) < geom.det_half[d])
    keys = philox.key64(n, t, c2, philox.STREAM_KEY_TRUE, seed)
    blk = vis["block"]

    p_list, b_list, gr_list, pl_list = [], [], [], []
    n_true = np.zeros(geom.n_blocks, dtype=np.int64)
    for b in range(geom.n_blocks):
        tt, dd = divmod(b, geom.n_det)
        sel = np.nonzero((blk == b) & keep)[0]
        n_true[b] = len(sel)
        n_out = int(np.floor(outlier_frac * len(sel) + 0.5))
        k = np.arange(n_out)
        u1, u2 = philox.uniforms2(k, tt, 65536 * dd, philox.STREAM_OUTLIER, seed)
        side = 2.0 * geom.det_half[dd]
        po = np.stack([(u1 - 0.5) * side, (u2 - 0.5) * side], axis=1)
        ko = philox.key64(k, tt, 65536 * dd, philox.STREAM_KEY_OUT, seed)
        allp = np.concatenate([s12[sel], po.reshape(-1, 2)])
        allk = np.concatenate([keys[sel], ko]).astype(np.uint64)
        src = np.concatenate([np.zeros(len(sel)), np.ones(n_out)])
        idx = np.concatenate([np.arange(len(sel)), k])
        order = np.lexsort((idx, src, allk))
        p_list.append(allp[order])
        b_list.append(np.full(len(order), b))
        gr = np.concatenate([n[sel], -np.ones(n_out, dtype=np.int64)])
        pl = np.concatenate([m[sel], -np.ones(n_out, dtype=np.int64)])
        gr_list.append(gr[order])
        pl_list.append(pl[order])
    block = np.concatenate(b_list).astype(np.int64)
    return {"p12": np.concatenate(p_list), "block": block,
            "offsets": forward.block_offsets(block, geom.n_blocks),
            "grain": np.concatenate(gr_list), "plane": np.concatenate(pl_list),
            "n_true": n_true}
