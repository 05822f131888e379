"""GPU parity of prototype scoring: pair candidates, single-grain refinement,
the unmatched filter, SPOT entries and greedy selection, against the oracle."""
import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import candidates, cost, crystal, forward, metrics, simulate, single

pytestmark = pytest.mark.gpu


def _setup(laue, n_rot=8, n_grains=12, sigma=1.0, frac=0.3, seed=11):
    p = ig.MEDIUM
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry(n_rot, np.deg2rad(180.0 / n_rot), p.detectors, p.lam_min, p.lam_max)
    q, x = ig.random_grains(p, n=n_grains, seed=seed)
    sim = simulate.simulate(pl, q, x, g, sigma, frac, seed, p.distance)
    p12 = ig.to_f32_exact(sim["p12"])
    geom = laue.make_geometry(n_rot, np.deg2rad(180.0 / n_rot), p.detectors, p.lam_min, p.lam_max)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    obs = laue.ObsSpots.from_numpy(p12, sim["offsets"])
    return p, pl, g, q, x, sim, p12, geom, planes, obs


def test_candidates_match_oracle(gpu_lib):
    laue = gpu_lib
    p, pl, g, q, x, sim, p12, geom, planes, obs = _setup(laue)
    ref = candidates.generate(pl, g, p12, sim["offsets"], 400, 77)
    gc = laue.laue_candidates_generate(geom, planes, obs, 400, 77)
    assert gc["n_found"] > 1000
    ko = set(zip(ref["pair"].tolist(), ref["ma"].tolist(), ref["mb"].tolist()))
    kg = set(zip(gc["pair"].cpu().tolist(), gc["ma"].cpu().tolist(), gc["mb"].cpu().tolist()))
    # hypotheses agree except at the angle-threshold edge (FP32 plane normals)
    diff = ko ^ kg
    assert len(diff) <= 2e-3 * len(ko), len(diff)
    idx = {k: i for i, k in enumerate(zip(ref["pair"].tolist(), ref["ma"].tolist(), ref["mb"].tolist()))}
    gi, oi = [], []
    for j, k in enumerate(zip(gc["pair"].cpu().tolist(), gc["ma"].cpu().tolist(), gc["mb"].cpu().tolist())):
        if k in idx:
            gi.append(j)
            oi.append(idx[k])
    qg = gc["q"].cpu().numpy()[gi]
    mis = np.degrees(metrics.misorientation(qg, ref["q"][oi]))
    assert np.max(mis) < 1e-4
    fg = gc["feat"].cpu().numpy()[gi][:, :14]
    assert np.allclose(fg, ref["feat"][oi], atol=2e-5)
    assert np.array_equal(gc["spot_a"].cpu().numpy()[gi], ref["a"][oi])


@pytest.mark.parametrize("drop_log2", [0.0, 26.0])
def test_refine_score_match_oracle(gpu_lib, drop_log2):
    """Refinement and scoring against the oracle (which keeps every pair), with
    the passes skipping only FP32-zero terms (0) and terms below 2^-26 of the
    outlier bin's (the default)."""
    laue = gpu_lib
    p, pl, g, q, x, sim, p12, geom, planes, obs = _setup(laue)
    ref = candidates.generate(pl, g, p12, sim["offsets"], 200, 5)
    mis = np.degrees(metrics.misorientation(ref["q"][:, None, :], q[None, :, :])).min(axis=1)
    # a few candidates near true grains, a few random ones
    sel = np.concatenate([np.argsort(mis)[:6], np.arange(0, len(mis), max(1, len(mis) // 6))[:6]])
    cq = ref["q"][sel]
    cx = np.zeros((len(sel), 3))
    c_out = cost.c_out(p.sigma_mm, p.distance)
    outs, slot_pairs = [], []
    n_obs_blk = np.diff(sim["offsets"])
    for k in range(len(sel)):
        qq, xx, mod = single.refine(pl, g, p.distance, p12, sim["offsets"], cq[k], cx[k], p.sigma_mm, c_out,
                                    k_refine=6, k_gn=2)
        slot_pairs.append(int(np.sum(np.diff(mod["offsets"]) * n_obs_blk)))
        outs.append((qq, xx) + single.score(pl, g, p.distance, p12, sim["offsets"], mod, qq, xx, p.sigma_mm, c_out))
    grains = laue.Grains(cq, cx)
    par = laue.score_params(p.sigma_mm, p.distance, c_out, k_refine=6, k_gn=2, chunk=5, drop_log2=drop_log2)
    res = laue.laue_score_candidates(geom, planes, obs, grains, par)
    qg, xg = grains.numpy()
    for k, (qq, xx, un, nm, rows, vals) in enumerate(outs):
        assert np.degrees(metrics.misorientation(qg[k], qq)) < 1e-3
        assert np.linalg.norm(xg[k] - xx) < 2e-3
        assert res["n_model"][k].item() == nm
        assert abs(res["n_unmatched"][k].item() - un) <= 1
        keep = nm > 0 and un < 0.1 * nm
        assert bool(res["keep"][k].item()) == keep
        lo, hi = res["lbar_off"][k].item(), res["lbar_off"][k + 1].item()
        if not keep:
            assert hi == lo
            continue
        gr = res["lbar_row"][lo:hi].cpu().numpy()
        gv = res["lbar_val"][lo:hi].cpu().numpy()
        phi = -c_out / (2 * p.sigma_mm ** 2)
        safe = np.abs(vals - phi) > 1e-3
        ro = set(rows[safe].tolist())
        assert ro <= set(gr.tolist())
        m = {r: v for r, v in zip(gr.tolist(), gv.tolist())}
        assert np.max(np.abs(np.array([m[r] for r in rows[safe]]) - vals[safe])) < 1e-4
    # at least some true-grain candidates survive the filter
    assert res["keep"].sum().item() >= 3
    # pairs streamed: 6 x 2 statistics passes and the first scoring pass over
    # every candidate's frozen model spots, the second over the kept ones
    kept = res["keep"].cpu().numpy().astype(bool)
    assert res["pairs_streamed"] == 13 * sum(slot_pairs) + sum(np.array(slot_pairs)[kept])
    # of those, the refinement passes' 12; the passes evaluate a part of them
    # (the refinement's within the zero radii, the scoring's within the
    # scoring radii)
    assert res["pairs_refine"] == 12 * sum(slot_pairs)
    assert 0 < res["pairs_evaluated"] <= res["pairs_streamed"]


@pytest.mark.parametrize("sigma", [1.0, 6.0])
def test_scoring_passes_match_oracle_dense(gpu_lib, sigma):
    """The scoring passes alone (k_refine = 0: the candidates, 8 true grains
    and 8 pair candidates, are scored where they start) on a dense sample (30
    grains, 70% outliers), against the oracle, which evaluates every pair.  At
    sigma = 6 mm the scoring radii
    (a few sigma) make the disks of a candidate's model spots of one block
    overlap, so rows are shared and taken by the slot's lowest-index spot.
    Unmatched counts, keep decisions and the SPOT entries (rows as a set,
    values) agree; a GPU entry missing from the oracle's set is at the floor
    within rounding."""
    laue = gpu_lib
    p, pl, g, q, x, sim, p12, geom, planes, obs = _setup(laue, n_grains=30, sigma=sigma, frac=0.7, seed=13)
    ref = candidates.generate(pl, g, p12, sim["offsets"], 200, 5)
    # 8 true grains (kept), 8 candidates spread over the list
    sel = np.arange(0, len(ref["q"]), max(1, len(ref["q"]) // 8))[:8]
    cq = np.concatenate([q[:8], ref["q"][sel]])
    cx = np.concatenate([x[:8], np.zeros((len(sel), 3))])
    c_out = cost.c_out(sigma, p.distance)
    par = laue.score_params(sigma, p.distance, c_out, k_refine=0, k_gn=1, chunk=7)
    res = laue.laue_score_candidates(geom, planes, obs, laue.Grains(cq, cx), par)
    phi = -c_out / (2 * sigma ** 2)
    close_pairs = 0
    for k in range(len(cq)):
        mod = forward.enumerate_visible(pl, cq[k][None], cx[k][None], g)
        mod["offsets"] = forward.block_offsets(mod["block"], g.n_blocks)
        un, nm, rows, vals = single.score(pl, g, p.distance, p12, sim["offsets"], mod, cq[k], cx[k], sigma, c_out)
        for b in range(g.n_blocks):
            s12 = mod["s12"][mod["offsets"][b]:mod["offsets"][b + 1]] if "s12" in mod else None
            if s12 is not None and len(s12) > 1:
                d = np.linalg.norm(s12[:, None, :] - s12[None, :, :], axis=-1)
                close_pairs += int(np.sum(np.triu(d < 6 * sigma, 1)))
        assert res["n_model"][k].item() == nm
        assert abs(res["n_unmatched"][k].item() - un) <= 1
        keep = nm > 0 and un < 0.1 * nm
        assert bool(res["keep"][k].item()) == keep
        lo, hi = res["lbar_off"][k].item(), res["lbar_off"][k + 1].item()
        if not keep:
            assert hi == lo
            continue
        gr = res["lbar_row"][lo:hi].cpu().numpy()
        gv = res["lbar_val"][lo:hi].cpu().numpy()
        assert len(set(gr.tolist())) == len(gr)             # each row once
        safe = np.abs(vals - phi) > 1e-3
        assert set(rows[safe].tolist()) <= set(gr.tolist())
        m = {r: v for r, v in zip(gr.tolist(), gv.tolist())}
        assert np.max(np.abs(np.array([m[r] for r in rows[safe]]) - vals[safe]), initial=0.0) < 1e-4
        extra = [v for r, v in m.items() if r not in set(rows.tolist())]
        assert all(abs(v - phi) < 1e-3 for v in extra)
    assert res["keep"].sum().item() >= 3
    if sigma > 2.0:
        assert close_pairs > 0


def test_greedy_matches_oracle(gpu_lib):
    laue = gpu_lib
    rng = np.random.default_rng(3)
    n_rows, n_cand, phi = 400, 30, -4.5
    cols = []
    for n in range(n_cand):
        r = np.sort(rng.choice(n_rows, size=rng.integers(5, 60), replace=False))
        v = phi + rng.uniform(0.01, 4.0, len(r))
        cols.append((r, v.astype(np.float32).astype(np.float64)))
    picks, gains = single.greedy(cols, n_rows, phi)
    off = np.concatenate([[0], np.cumsum([len(c[0]) for c in cols])])
    rows = np.concatenate([c[0] for c in cols]).astype(np.int32)
    vals = np.concatenate([c[1] for c in cols]).astype(np.float32)
    dev = torch.device("cuda")
    gp, gg = laue.laue_spot_greedy(torch.tensor(off, device=dev), torch.tensor(rows, device=dev),
                                   torch.tensor(vals, device=dev), n_cand, n_rows, phi, n_cand)
    assert gp.cpu().tolist() == picks
    assert np.allclose(gg.cpu().numpy(), gains, rtol=1e-9, atol=1e-9)
    assert single.n_prototypes(gg.cpu().numpy()) == single.n_prototypes(gains)


@pytest.mark.parametrize("compact", [True, False])
def test_band_greedy_matches_oracle_many_candidates(gpu_lib, compact):
    """Hundreds of overlapping candidates, exact duplicates among them (ties
    go to the lowest index): the band steps (stale increments as upper
    bounds) pick exactly what the plain greedy picks, with the same gains."""
    laue = gpu_lib
    rng = np.random.default_rng(11)
    n_rows, phi = 3000, -4.5
    cols = []
    for n in range(300):
        centre = rng.integers(0, n_rows)
        r = np.unique(np.clip(centre + rng.integers(-150, 150, size=rng.integers(10, 120)), 0, n_rows - 1))
        v = phi + rng.uniform(0.01, 4.0, len(r))
        cols.append((r, v.astype(np.float32).astype(np.float64)))
    for n in rng.choice(300, size=30, replace=False):
        cols.append((cols[n][0].copy(), cols[n][1].copy()))
    k_max = 150
    picks, gains = single.greedy(cols, n_rows, phi, k_max)
    off = np.concatenate([[0], np.cumsum([len(c[0]) for c in cols])])
    rows = np.concatenate([c[0] for c in cols]).astype(np.int32)
    vals = np.concatenate([c[1] for c in cols]).astype(np.float32)
    dev = torch.device("cuda")
    gp, gg = laue.laue_spot_greedy(torch.tensor(off, device=dev), torch.tensor(rows, device=dev),
                                   torch.tensor(vals, device=dev), len(cols), n_rows, phi, k_max, compact=compact)
    assert gp.cpu().tolist() == picks
    assert np.allclose(gg.cpu().numpy(), gains, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("compact", [True, False])
def test_greedy_heavy_overlap_matches_oracle(gpu_lib, compact):
    """Every candidate covers a third of the rows, as under dense clutter: each
    pick lowers almost every other gain, so most bounds go stale at every step
    and the band steps recompute many of them; the picks and gains stay those
    of the plain greedy."""
    laue = gpu_lib
    rng = np.random.default_rng(5)
    n_rows, n_cand, phi, k_max = 2000, 400, -4.5, 120
    cols = []
    for n in range(n_cand):
        r = np.sort(rng.choice(n_rows, size=rng.integers(500, 700), replace=False))
        v = phi + rng.uniform(0.01, 4.0, len(r))
        cols.append((r, v.astype(np.float32).astype(np.float64)))
    cols.append((cols[7][0].copy(), cols[7][1].copy()))          # an exact duplicate: the lower index wins
    picks, gains = single.greedy(cols, n_rows, phi, k_max)
    off = np.concatenate([[0], np.cumsum([len(c[0]) for c in cols])])
    rows = np.concatenate([c[0] for c in cols]).astype(np.int32)
    vals = np.concatenate([c[1] for c in cols]).astype(np.float32)
    dev = torch.device("cuda")
    gp, gg = laue.laue_spot_greedy(torch.tensor(off, device=dev), torch.tensor(rows, device=dev),
                                   torch.tensor(vals, device=dev), len(cols), n_rows, phi, k_max, compact=compact)
    assert gp.cpu().tolist() == picks
    assert np.allclose(gg.cpu().numpy(), gains, rtol=1e-9, atol=1e-9)


def test_greedy_ends_early(gpu_lib):
    """Two hundred copies of one column and three small disjoint columns: after
    the first pick every copy's increment is zero (their stale bounds are
    recomputed to 0), the three others are picked and the selection stops with
    no positive increment left (fewer picks than k_max)."""
    laue = gpu_lib
    rng = np.random.default_rng(9)
    n_rows, phi = 1200, -4.5
    base_r = np.sort(rng.choice(1000, size=600, replace=False))
    base_v = (phi + rng.uniform(0.5, 4.0, len(base_r))).astype(np.float32).astype(np.float64)
    cols = [(base_r.copy(), base_v.copy()) for _ in range(200)]
    for k in range(3):
        r = np.arange(1000 + 60 * k, 1000 + 60 * k + 40)
        cols.append((r, (phi + rng.uniform(0.01, 1.0, len(r))).astype(np.float32).astype(np.float64)))
    picks, gains = single.greedy(cols, n_rows, phi, 50)
    assert len(picks) == 4
    off = np.concatenate([[0], np.cumsum([len(c[0]) for c in cols])])
    rows = np.concatenate([c[0] for c in cols]).astype(np.int32)
    vals = np.concatenate([c[1] for c in cols]).astype(np.float32)
    dev = torch.device("cuda")
    gp, gg = laue.laue_spot_greedy(torch.tensor(off, device=dev), torch.tensor(rows, device=dev),
                                   torch.tensor(vals, device=dev), len(cols), n_rows, phi, 50)
    assert gp.cpu().tolist() == picks
    assert np.allclose(gg.cpu().numpy(), gains, rtol=1e-9, atol=1e-9)


def test_greedy_many_candidates_exact_increments(gpu_lib):
    """300,000 small candidates in clusters of shared rows (more than one pass
    of the scan and recompute grids), exact duplicates among them, values on a
    1/8 grid so that every increment is exact in any summation order: each
    pick is the lowest-index candidate of largest increment, the increments
    recomputed here from the definition of the set function at every step."""
    laue = gpu_lib
    rng = np.random.default_rng(21)
    n_rows, n_cand, phi, k_max = 20000, 300_000, -4.5, 40
    centre = rng.integers(0, n_rows, size=n_cand)
    cnt = rng.integers(1, 9, size=n_cand)
    off = np.concatenate([[0], np.cumsum(cnt)])
    seg = np.repeat(np.arange(n_cand), cnt)
    rows = np.clip(centre[seg] + rng.integers(-40, 40, size=off[-1]), 0, n_rows - 1)
    vals = phi + rng.integers(1, 33, size=off[-1]) / 8.0
    for c in rng.choice(n_cand - 1, size=2000, replace=False):    # duplicate c into c + 1
        if cnt[c] == cnt[c + 1]:
            rows[off[c + 1]:off[c + 2]] = rows[off[c]:off[c + 1]]
            vals[off[c + 1]:off[c + 2]] = vals[off[c]:off[c + 1]]
    # a candidate holds at most one entry per row: keep the first of repeats
    keep = np.ones(off[-1], bool)
    for c in range(n_cand):
        r = rows[off[c]:off[c + 1]]
        _, first = np.unique(r, return_index=True)
        k = np.zeros(len(r), bool)
        k[first] = True
        keep[off[c]:off[c + 1]] = k
    rows, vals, seg = rows[keep], vals[keep], seg[keep]
    cnt = np.bincount(seg, minlength=n_cand)
    off = np.concatenate([[0], np.cumsum(cnt)])
    cur = np.full(n_rows, phi)
    picked = np.zeros(n_cand, bool)
    picks, gains = [], []
    for _ in range(k_max):
        inc = np.bincount(seg, weights=np.maximum(0.0, vals - cur[rows]), minlength=n_cand)
        inc[picked] = -1.0
        c = int(np.argmax(inc))                 # the first of equal maxima
        if inc[c] <= 0.0:
            break
        picks.append(c)
        gains.append(inc[c])
        picked[c] = True
        r = rows[off[c]:off[c + 1]]
        cur[r] = np.maximum(cur[r], vals[off[c]:off[c + 1]])
    dev = torch.device("cuda")
    gp, gg = laue.laue_spot_greedy(torch.tensor(off, device=dev), torch.tensor(rows.astype(np.int32), device=dev),
                                   torch.tensor(vals.astype(np.float32), device=dev), n_cand, n_rows, phi, k_max)
    assert gp.cpu().tolist() == picks
    assert np.array_equal(gg.cpu().numpy(), np.array(gains))
