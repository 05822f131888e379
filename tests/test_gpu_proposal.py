"""GPU parity of the learned proposal's support features, labels and
top-fraction selection against the oracle; properties at full size."""
import math

import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import candidates, crystal, forward, metrics, proposal, simulate

pytestmark = pytest.mark.gpu


def _setup(laue, n_rot=12, n_grains=20, sigma=1.0, frac=0.3, seed=21):
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


def _upload(ref):
    dev = "cuda"
    n = len(ref["q"])
    return {"q": torch.tensor(ref["q"], dtype=torch.float64, device=dev),
            "spot_a": torch.tensor(ref["a"], dtype=torch.int32, device=dev),
            "spot_b": torch.tensor(ref["b"], dtype=torch.int32, device=dev),
            "feat": torch.zeros((max(n, 1), 16), dtype=torch.float32, device=dev)[:n]}


@pytest.mark.parametrize("radius", [1.0, 3.0])
def test_support_matches_oracle(gpu_lib, radius):
    laue = gpu_lib
    p, pl, g, q, x, sim, p12, geom, planes, obs = _setup(laue)
    ref = candidates.generate(pl, g, p12, sim["offsets"], 150, 31)
    n = len(ref["q"])
    assert n > 500
    c = _upload(ref)
    n_sup = len(pl["d"])
    laue.laue_candidate_support(geom, planes, obs, c, radius, n_sup)
    fg = c["feat"].cpu().numpy()[:, 14:16]
    # sampled candidates (the oracle is a per-plane Python loop), plus the ragged end
    idx = np.unique(np.concatenate([np.arange(0, n, max(1, n // 120)), np.arange(n - 5, n)]))
    t_pair = np.searchsorted(sim["offsets"], ref["a"][idx], side="right") - 1
    fo, border = proposal.support(pl, g, p12, sim["offsets"], ref["q"][idx], t_pair // g.n_det, radius, n_sup)
    npred = np.array([[len(proposal.predict(pl, g, crystal.quat_to_R(ref["q"][i]), t,
                                            proposal.probe_planes(pl, n_sup)))
                       for t in proposal.probe_rotations(int(tp // g.n_det), g.n_rot)]
                      for i, tp in zip(idx, t_pair)])
    tol = border[:, None] / np.maximum(npred, 1) + 1e-7
    assert np.all(np.abs(fg[idx] - fo) <= tol)
    assert np.mean(fo > 0) > 0.05          # the check is not vacuous


def test_support_true_grains_full_size(gpu_lib):
    laue = gpu_lib
    p = ig.LEARNED
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    q, x = ig.random_grains(p, n=p.n_grains, seed=p.seed)
    truth = laue.Grains(q, np.zeros_like(x))
    obs = laue.laue_simulate(geom, planes, truth, 0.0, p.distance, p.outlier_frac, p.seed)
    gr = obs.grain.cpu().numpy()
    # each true grain as a candidate, its pair spot the first detected spot of that grain
    first = np.full(len(q), -1)
    for i in range(len(gr) - 1, -1, -1):
        if gr[i] >= 0:
            first[gr[i]] = i
    ok = first >= 0
    dev = "cuda"
    c = {"q": torch.tensor(q[ok], device=dev), "spot_a": torch.tensor(first[ok], dtype=torch.int32, device=dev),
         "feat": torch.zeros((int(ok.sum()), 16), dtype=torch.float32, device=dev)}
    laue.laue_candidate_support(geom, planes, obs, c, 1.0, planes.n)
    f = c["feat"].cpu().numpy()[:, 14:16]
    assert np.all(f == 1.0)
    # random orientations are hit only by chance
    qr = ig.random_quaternions(np.random.default_rng(99), 4096)
    c = {"q": torch.tensor(qr, device=dev),
         "spot_a": torch.tensor(np.arange(4096) * 37 % obs.n, dtype=torch.int32, device=dev),
         "feat": torch.zeros((4096, 16), dtype=torch.float32, device=dev)}
    laue.laue_candidate_support(geom, planes, obs, c, 1.0, planes.n)
    fr = c["feat"].cpu().numpy()[:, 14:16]
    assert fr.mean() < 0.9


def test_labels_match_oracle(gpu_lib):
    laue = gpu_lib
    p, pl, g, q, x, sim, p12, geom, planes, obs = _setup(laue, n_grains=6, seed=5)
    ref = candidates.generate(pl, g, p12, sim["offsets"], 400, 3)
    lab_o, mis_o = proposal.labels(ref["q"], ref["a"], ref["b"], sim["grain"], q)
    assert lab_o.sum() >= 5
    c = _upload(ref)
    truth = laue.Grains(q, x)
    lab_g, mis_g = laue.laue_candidate_labels(c, torch.tensor(sim["grain"], dtype=torch.int32, device="cuda"),
                                              truth, 2.0)
    lab_g, mis_g = lab_g.cpu().numpy(), mis_g.cpu().numpy()
    fin = np.isfinite(mis_o)
    assert np.array_equal(np.isfinite(mis_g), fin)
    assert np.allclose(mis_g[fin], mis_o[fin], atol=1e-4)
    edge = np.abs(mis_o - 2.0) < 1e-6
    assert np.array_equal(lab_g[~edge], lab_o[~edge])


def test_nearest_labels_match_oracle(gpu_lib):
    """Labels by the nearest true grain on candidates of random pairs and on
    orientations placed near the true grains (so that both labels occur)."""
    laue = gpu_lib
    p, pl, g, q, x, sim, p12, geom, planes, obs = _setup(laue, n_grains=6, seed=5)
    ref = candidates.generate(pl, g, p12, sim["offsets"], 400, 3)
    rng = np.random.default_rng(4)
    ang = np.radians(rng.uniform(0.0, 2.0, 60))
    ax = rng.standard_normal((60, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    dq = np.concatenate([np.cos(ang / 2)[:, None], np.sin(ang / 2)[:, None] * ax], axis=1)
    base = q[rng.integers(0, len(q), 60)]
    w0, x0, y0, z0 = base.T
    w1, x1, y1, z1 = dq.T
    near_q = np.stack([w0 * w1 - x0 * x1 - y0 * y1 - z0 * z1, w0 * x1 + x0 * w1 + y0 * z1 - z0 * y1,
                       w0 * y1 - x0 * z1 + y0 * w1 + z0 * x1, w0 * z1 + x0 * y1 - y0 * x1 + z0 * w1], axis=1)
    cq = np.concatenate([ref["q"], near_q])
    lab_o, mis_o, near_o = proposal.labels_nearest(cq, q, 1.0)
    assert 10 <= lab_o.sum() < len(cq)
    c = {"q": torch.tensor(cq, device="cuda")}
    lab_g, mis_g, near_g = laue.laue_candidate_labels_nearest(c, laue.Grains(q, x), 1.0)
    lab_g, mis_g, near_g = lab_g.cpu().numpy(), mis_g.cpu().numpy(), near_g.cpu().numpy()
    assert np.allclose(mis_g, mis_o, atol=1e-4)
    edge = np.abs(mis_o - 1.0) < 1e-6
    assert np.array_equal(lab_g[~edge], lab_o[~edge])
    # the nearest grain where it is unique (no other grain within 1e-6 deg)
    all_mis = np.degrees(metrics.misorientation(cq[:, None, :], q[None, :, :]))
    second = np.sort(all_mis, axis=1)[:, 1] if len(q) > 1 else np.full(len(cq), np.inf)
    uniq = second - mis_o > 1e-6
    assert np.array_equal(near_g[uniq], near_o[uniq])


@pytest.mark.parametrize("n,frac", [(1, 1.0), (7, 0.5), (1000, 0.05), (100003, 0.05), (262144, 0.3)])
def test_select_top_matches_oracle(gpu_lib, n, frac):
    laue = gpu_lib
    rng = np.random.default_rng(n)
    s = rng.integers(0, 50, n).astype(np.float32) / 49.0        # many ties
    s[rng.integers(0, n, max(1, n // 100))] = -rng.uniform(0, 1, max(1, n // 100)).astype(np.float32)
    k = min(n, math.ceil(frac * n))
    got = laue.laue_select_top(torch.tensor(s, device="cuda"), k).cpu().numpy()
    want = proposal.select_top(s.astype(np.float64), frac)
    assert np.array_equal(got, want)


def test_select_top_edge_cases(gpu_lib):
    laue = gpu_lib
    s = torch.tensor([0.5, float("nan"), 0.5, -0.0, 0.0, 1.0], device="cuda")
    assert laue.laue_select_top(s, 0).numel() == 0
    assert laue.laue_select_top(s, 6).cpu().tolist() == [0, 1, 2, 3, 4, 5]
    assert laue.laue_select_top(s, 3).cpu().tolist() == [0, 2, 5]
    # -0.0 equals +0.0 (taken by index); NaN last
    assert laue.laue_select_top(s, 4).cpu().tolist() == [0, 2, 3, 5]
    assert laue.laue_select_top(s, 5).cpu().tolist() == [0, 2, 3, 4, 5]
    # full size: a property check on 2^20 scores
    n = 1 << 20
    v = torch.rand(n, device="cuda")
    k = math.ceil(0.05 * n)
    idx = laue.laue_select_top(v, k)
    assert idx.numel() == k and bool((idx[1:] > idx[:-1]).all())
    chosen = torch.zeros(n, dtype=torch.bool, device="cuda")
    chosen[idx.long()] = True
    assert v[chosen].min().item() >= v[~chosen].max().item()


def test_same_grain_pairs_and_explicit_candidates(gpu_lib):
    laue = gpu_lib
    p, pl, g, q, x, sim, p12, geom, planes, obs = _setup(laue, n_grains=10, seed=8)
    a_o, b_o = proposal.same_grain_pairs(sim["offsets"], sim["grain"], g.n_det, 3000, 77)
    gr = torch.tensor(sim["grain"], dtype=torch.int32, device="cuda")
    a_g, b_g = laue.laue_pairs_same_grain(geom, obs, gr, 3000, 77)
    assert np.array_equal(a_g.cpu().numpy(), a_o) and np.array_equal(b_g.cpu().numpy(), b_o)
    # candidates of explicit pairs (a few invalid ones mixed in)
    a_e = a_o[:120].copy()
    b_e = b_o[:120].copy()
    a_e[5], b_e[7] = len(p12) + 3, -4
    ref = candidates.generate(pl, g, p12, sim["offsets"], 0, 0, pairs=(a_e, b_e))
    pa = torch.tensor(a_e, dtype=torch.int32, device="cuda")
    pb = torch.tensor(b_e, dtype=torch.int32, device="cuda")
    gc = laue.laue_candidates_generate(geom, planes, obs, 0, 0, pairs=(pa, pb))
    ko = list(zip(ref["pair"].tolist(), ref["ma"].tolist(), ref["mb"].tolist()))
    kg = list(zip(gc["pair"].cpu().tolist(), gc["ma"].cpu().tolist(), gc["mb"].cpu().tolist()))
    assert len(ko) > 300
    assert len(set(ko) ^ set(kg)) <= 2e-3 * len(ko)
    lab, _ = proposal.labels(ref["q"], ref["a"], ref["b"], sim["grain"], q)
    assert lab.mean() > 0.02            # same-grain pairs carry positives
