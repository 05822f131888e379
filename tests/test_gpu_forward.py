"""GPU parity of the forward model and the simulator against the oracle."""
import dataclasses

import numpy as np
import pytest

import inputgen as ig
from oracle import cost, crystal, forward, simulate

pytestmark = pytest.mark.gpu


def _setup(laue, preset, n_rot=None, n_grains=None):
    p = preset
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry(p.n_rot if n_rot is None else n_rot, np.deg2rad(p.domega_deg), p.detectors,
                         p.lam_min, p.lam_max)
    q, x = ig.random_grains(p, n=n_grains)
    geom = laue.make_geometry(g.n_rot, np.deg2rad(p.domega_deg), p.detectors, p.lam_min, p.lam_max)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    return pl, g, q, x, geom, planes


def _compare_sets(V, M, n_det, merge):
    """Index sets equal except items the oracle flags as within the edge margins."""
    o = set(zip(V["t"].tolist(), V["det"].tolist(), V["n"].tolist(), V["m"].tolist()))
    g = set(zip((M["block"] // n_det).tolist(), (M["block"] % n_det).tolist(), M["grain"].tolist(),
                M["plane"].tolist()))
    flagged = {k for k, f in zip(zip(V["t"].tolist(), V["det"].tolist(), V["n"].tolist(),
                                     V["m"].tolist()), V["flag"]) if f}
    flagged |= {(t, d, n, m) for (n, t, m, d) in V["near_edge"]}
    gflag = {k for k, f in zip(zip((M["block"] // n_det).tolist(), (M["block"] % n_det).tolist(),
                                   M["grain"].tolist(), M["plane"].tolist()), M["flags"]) if f}
    diff = (o ^ g) - flagged - gflag
    assert not diff, f"{len(diff)} unflagged differences, e.g. {sorted(diff)[:5]}"
    return o & g


@pytest.mark.parametrize("name,n_rot,n_grains,merge", [("tiny", None, None, True),
                                                       ("tiny", None, None, False),
                                                       ("medium", None, None, True),
                                                       ("medium", 7, 40, False),
                                                       ("stress", 5, 60, True)])
def test_enumerate_matches_oracle(gpu_lib, name, n_rot, n_grains, merge):
    laue = gpu_lib
    pl, g, q, x, geom, planes = _setup(laue, ig.PRESETS[name], n_rot, n_grains)
    V = forward.enumerate_visible(pl, q, x, g, merge_harmonics=merge)
    M = laue.laue_forward_enumerate(geom, planes, laue.Grains(q, x), merge).numpy()
    common = _compare_sets(V, M, g.n_det, merge)
    assert len(common) > 0.99 * len(V["m"])
    # order (t, d, n, m) and block offsets
    key = M["block"].astype(np.int64) * 10**9 + M["grain"].astype(np.int64) * 10**4 + M["plane"]
    assert np.all(np.diff(key) > 0)
    assert np.array_equal(M["block_off"], np.concatenate([[0], np.cumsum(np.bincount(M["block"], minlength=g.n_blocks))]))
    # positions and wavelengths of common items
    idx = {k: i for i, k in enumerate(zip(V["t"].tolist(), V["det"].tolist(), V["n"].tolist(), V["m"].tolist()))}
    gi, oi = [], []
    for j, k in enumerate(zip((M["block"] // g.n_det).tolist(), (M["block"] % g.n_det).tolist(),
                              M["grain"].tolist(), M["plane"].tolist())):
        if k in idx:
            gi.append(j)
            oi.append(idx[k])
    gi, oi = np.array(gi), np.array(oi)
    assert np.max(np.abs(M["s1"][gi] - V["s12"][oi, 0])) < 2e-3
    assert np.max(np.abs(M["s2"][gi] - V["s12"][oi, 1])) < 2e-3
    assert np.max(np.abs(M["lam"][gi] - V["lam"][oi]) / V["lam"][oi]) < 1e-6
    ev = forward.eval_fixed(pl, q, x, g, V["m"][oi], V["n"][oi], V["t"][oi], V["det"][oi])
    vl = cost.v_local(g, V["det"][oi], ev["v"])
    for c, col in enumerate(("vn", "v1", "v2")):
        assert np.max(np.abs(M[col][gi] - vl[:, c])) < 2e-3


# Many planes (868, 28 mask words per detector), a wide band and large
# detectors close to the sample: about 4,300 kept spots per 16-grain work item
# of the write pass, so its LDS list (2048 entries) is written out in the
# middle of a detector's run, and the mask words exceed what it prefetches.
WIDE = dataclasses.replace(
    ig.STRESS, a=4.05, centering="F", n_max=84, lam_min=0.2, lam_max=8.0,
    detectors=(ig.Detector((30.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), 500.0),
               ig.Detector((-30.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), 500.0)))


@pytest.mark.parametrize("merge", [True, False])
def test_enumerate_long_lists_match_oracle(gpu_lib, merge):
    laue = gpu_lib
    pl, g, q, x, geom, planes = _setup(laue, WIDE, 3, 40)      # 40 grains: chunks of 16, 16 and 8
    V = forward.enumerate_visible(pl, q, x, g, merge_harmonics=merge)
    # more than 2048 kept spots per 16 grains and rotation (both detectors)
    assert np.bincount(V["t"]).min() * 16 / 40 > 2048
    M = laue.laue_forward_enumerate(geom, planes, laue.Grains(q, x), merge).numpy()
    common = _compare_sets(V, M, g.n_det, merge)
    assert len(common) > 0.99 * len(V["m"])
    key = M["block"].astype(np.int64) * 10**9 + M["grain"].astype(np.int64) * 10**4 + M["plane"]
    assert np.all(np.diff(key) > 0)
    assert np.array_equal(M["block_off"], np.concatenate([[0], np.cumsum(np.bincount(M["block"], minlength=g.n_blocks))]))


def test_enumerate_candidate_scale_equals_eval(gpu_lib):
    """8192 grains of the 1000-grain workload's lattice, band and 60-rotation
    scan: the write pass's geometry equals, bit for bit, the frozen-list
    evaluation of the ids it wrote (one forward model, two kernels), and the
    ids are in (block, grain, plane) order with matching block offsets."""
    laue = gpu_lib
    p = ig.LEARNED
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    q, x = ig.random_grains(p, n=8192, seed=p.seed + 11)
    M = laue.laue_forward_enumerate(geom, planes, laue.Grains(q, x), True)
    A = M.numpy()
    assert M.n > 1_000_000
    key = A["block"].astype(np.int64) * 10**9 + A["grain"].astype(np.int64) * 10**4 + A["plane"]
    assert np.all(np.diff(key) > 0)
    nb = len(A["block_off"]) - 1
    assert np.array_equal(A["block_off"], np.concatenate([[0], np.cumsum(np.bincount(A["block"], minlength=nb))]))
    E = laue.ModelSpots.from_arrays(nb, A["block_off"], A["plane"], A["grain"], A["block"])
    laue.laue_forward_eval(geom, planes, laue.Grains(q, x), E)
    B = E.numpy()
    for f in ("s1", "s2", "vn", "v1", "v2", "lam"):
        assert np.array_equal(A[f].view(np.uint32), B[f].view(np.uint32)), f


def test_enumerate_counted_equals_one_call(gpu_lib):
    """laue_forward_enumerate_counted after a capacity query writes, bit for
    bit, what one laue_forward_enumerate call with room writes; it refuses a
    workspace with no count, changed arguments and a short capacity."""
    import ctypes as C
    laue = gpu_lib
    lib = laue.require_native()
    pl, g, q, x, geom, planes = _setup(laue, ig.MEDIUM, 7, 40)
    grains = laue.Grains(q, x)
    nb = laue.n_blocks(geom)
    wsz = lib.laue_forward_workspace_size(C.byref(geom), planes.n, grains.n)
    ws = laue._workspace(wsz)
    n = laue.laue_forward_count(geom, planes, grains, True)
    assert n > 1000
    stream = laue._stream()

    def call(fn, out, merge=1, ws_=ws, cap=None):
        st = out.struct()
        if cap is not None:
            st.n = cap
        nout = C.c_int64()
        rc = fn(C.byref(geom), C.byref(planes.struct), C.byref(grains.struct), merge, C.byref(st), C.byref(nout),
                laue._ptr(ws_), ws_.numel(), stream)
        return rc, nout.value

    A = laue.ModelSpots(n, nb)
    assert call(lib.laue_forward_enumerate, A) == (0, n)
    # a capacity query, then the counted write
    assert call(lib.laue_forward_enumerate, laue.ModelSpots(0, nb), cap=0) == (laue._abi.LAUE_ECAPACITY, n)
    B = laue.ModelSpots(n, nb)
    assert call(lib.laue_forward_enumerate_counted, B) == (0, n)
    a, b = A.numpy(), B.numpy()
    for f in a:
        assert np.array_equal(a[f].view(np.uint8), b[f].view(np.uint8)), f
    # the same count serves again; a short capacity is refused with the size
    assert call(lib.laue_forward_enumerate_counted, laue.ModelSpots(n, nb))[0] == 0
    assert call(lib.laue_forward_enumerate_counted, laue.ModelSpots(n - 1, nb)) == (laue._abi.LAUE_ECAPACITY, n)
    # other arguments, or a workspace that holds no count
    assert call(lib.laue_forward_enumerate_counted, laue.ModelSpots(n, nb), merge=0)[0] == laue._abi.LAUE_EINVAL
    other = laue._workspace(wsz + 4096)
    assert call(lib.laue_forward_enumerate_counted, laue.ModelSpots(n, nb), ws_=other)[0] == laue._abi.LAUE_EINVAL
    # a workspace overwritten since the count
    ws.fill_(0)
    assert call(lib.laue_forward_enumerate_counted, laue.ModelSpots(n, nb))[0] == laue._abi.LAUE_EINVAL


def test_enumerate_empty_and_capacity(gpu_lib):
    laue = gpu_lib
    pl, g, q, x, geom, planes = _setup(laue, ig.TINY)
    M = laue.laue_forward_enumerate(geom, planes, laue.Grains(np.zeros((0, 4)), np.zeros((0, 3))))
    assert M.n == 0 and np.all(M.block_off == 0)


def test_eval_matches_oracle(gpu_lib):
    laue = gpu_lib
    pl, g, q, x, geom, planes = _setup(laue, ig.MEDIUM, 9, 30)
    S = forward.enumerate_visible(pl, q, x, g)
    q2, x2 = ig.perturb_grains(q, x, 0.7, 0.4, 5)
    M = laue.ModelSpots.from_arrays(g.n_blocks, forward.block_offsets(S["block"], g.n_blocks),
                                    S["m"], S["n"], S["block"])
    laue.laue_forward_eval(geom, planes, laue.Grains(q2, x2), M)
    Mg = M.numpy()
    ev = forward.eval_fixed(pl, q2, x2, g, S["m"], S["n"], S["t"], S["det"])
    vl = cost.v_local(g, S["det"], ev["v"])
    assert np.max(np.abs(Mg["s1"] - ev["s12"][:, 0])) < 2e-3
    assert np.max(np.abs(Mg["s2"] - ev["s12"][:, 1])) < 2e-3
    for c, col in enumerate(("vn", "v1", "v2")):
        assert np.max(np.abs(Mg[col] - vl[:, c])) < 2e-3


@pytest.mark.parametrize("name,n_rot,n_grains", [("tiny", None, None), ("medium", 6, 50)])
def test_simulate_matches_oracle(gpu_lib, name, n_rot, n_grains):
    laue = gpu_lib
    p = ig.PRESETS[name]
    pl, g, q, x, geom, planes = _setup(laue, p, n_rot, n_grains)
    sim = simulate.simulate(pl, q, x, g, p.sigma_mm, p.outlier_frac, p.seed, p.distance)
    ob = laue.laue_simulate(geom, planes, laue.Grains(q, x), p.sigma_mm, p.distance, p.outlier_frac, p.seed)
    assert np.array_equal(ob.block_off, sim["offsets"])
    n = ob.n
    p1 = ob.p1[:n].cpu().numpy()
    p2 = ob.p2[:n].cpu().numpy()
    assert np.array_equal(ob.grain[:n].cpu().numpy(), sim["grain"])
    assert np.array_equal(ob.plane[:n].cpu().numpy(), sim["plane"])
    assert np.max(np.abs(p1 - sim["p12"][:, 0])) < 1e-3
    assert np.max(np.abs(p2 - sim["p12"][:, 1])) < 1e-3
