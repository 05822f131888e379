"""Full-size checks at the workloads the bench times: sampled outputs the
oracle computes one by one, and properties that hold at any size."""
import math

import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import crystal, forward, mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n_sample", [("learned", 6), ("stress", 4)])
def test_forward_full_size_sampled_grains(gpu_lib, name, n_sample):
    laue = gpu_lib
    p = ig.PRESETS[name]
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry.from_preset(p)
    q, x = ig.random_grains(p)
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    M = laue.laue_forward_enumerate(geom, planes, laue.Grains(q, x), True).numpy()
    sample = np.random.default_rng(3).choice(len(q), n_sample, replace=False)
    V = forward.enumerate_visible(pl, q[sample], x[sample], g, merge_harmonics=True)
    V["n"] = sample[V["n"]]
    V["near_edge"] = [(int(sample[n]), t, m, d) for (n, t, m, d) in V["near_edge"]]
    sel = np.isin(M["grain"], sample)
    Ms = {k: (v[sel] if isinstance(v, np.ndarray) and len(v) == len(sel) else v) for k, v in M.items()}
    o = set(zip(V["t"].tolist(), V["det"].tolist(), V["n"].tolist(), V["m"].tolist()))
    gs = set(zip((Ms["block"] // g.n_det).tolist(), (Ms["block"] % g.n_det).tolist(), Ms["grain"].tolist(),
                 Ms["plane"].tolist()))
    flagged = {k for k, f in zip(zip(V["t"].tolist(), V["det"].tolist(), V["n"].tolist(), V["m"].tolist()),
                                 V["flag"]) if f}
    flagged |= {(t, d, n, m) for (n, t, m, d) in V["near_edge"]}
    gflag = {k for k, f in zip(zip((Ms["block"] // g.n_det).tolist(), (Ms["block"] % g.n_det).tolist(),
                                   Ms["grain"].tolist(), Ms["plane"].tolist()), Ms["flags"]) if f}
    assert not ((o ^ gs) - flagged - gflag)
    assert len(o) > 100 * n_sample
    idx = {k: i for i, k in enumerate(zip(V["t"].tolist(), V["det"].tolist(), V["n"].tolist(), V["m"].tolist()))}
    gi = [j for j, k in enumerate(zip((Ms["block"] // g.n_det).tolist(), (Ms["block"] % g.n_det).tolist(),
                                      Ms["grain"].tolist(), Ms["plane"].tolist())) if k in idx]
    oi = [idx[(int(Ms["block"][j] // g.n_det), int(Ms["block"][j] % g.n_det), int(Ms["grain"][j]),
               int(Ms["plane"][j]))] for j in gi]
    assert np.max(np.abs(Ms["s1"][gi] - V["s12"][oi, 0])) < 2e-3
    assert np.max(np.abs(Ms["s2"][gi] - V["s12"][oi, 1])) < 2e-3


def test_sinkhorn_full_size_marginals(gpu_lib):
    """1000 grains, 70% outliers: after convergence from zero potentials every
    sampled row of the plan (with its outlier entry) and every sampled column
    (with its unmatched entry) sums to one."""
    laue = gpu_lib
    p = ig.LEARNED
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    q, x = ig.random_grains(p)
    obs = laue.laue_simulate(geom, planes, laue.Grains(q, x), p.sigma_mm, p.distance, p.outlier_frac, p.seed)
    q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, p.seed + 17)
    model = laue.laue_forward_enumerate(geom, planes, laue.Grains(q0, x0), True)
    c_out = 2.0 * p.distance ** 2 * (1.0 - math.cos(3.0 * p.sigma_mm / p.distance))
    eps = p.eps_start
    t_b = float(math.ceil(0.4 * model.n))
    ot = laue.ot_params(eps, p.distance, c_out, t_b, tol=1e-5, n_max=2000)
    f = torch.zeros(obs.n, dtype=torch.float32, device="cuda")
    g = torch.zeros(model.n, dtype=torch.float32, device="cuda")
    f0, g0, st, rc = laue.laue_sinkhorn(geom, obs, model, ot, f, g)
    assert st["converged"] and st["err"] <= 4e-5
    nI = np.diff(obs.block_off)
    nJ = np.diff(model.block_off)
    blocks = [int(np.argmax(nI * nJ)), int(np.argmin(np.where(nI * nJ > 0, nI * nJ, np.inf))), 37]
    fc, gc = f.double().cpu().numpy(), g.double().cpu().numpy()
    for b in blocks:
        Q = laue.laue_plan_block(geom, obs, model, ot, f, g, b).double().cpu().numpy()
        r0, c0 = obs.block_off[b], model.block_off[b]
        q_out = np.exp((fc[r0:r0 + nI[b]] + g0 - c_out) / eps)
        q_unm = np.exp((f0 + gc[c0:c0 + nJ[b]] - 0.0) / eps)
        assert np.max(np.abs(Q.sum(axis=1) + q_out - 1.0)) < 1e-4
        assert np.max(np.abs(Q.sum(axis=0) + q_unm - 1.0)) < 1e-4
        assert Q.min() >= 0.0 and Q.max() <= 1.0 + 1e-6


def test_cold_stage_converges_full_size(gpu_lib):
    """1000 grains, 70% outliers: the EM runs the schedule 111 -> 3.51 sigma^2
    (16 iterations), then a Sinkhorn at the last temperature 1.11 sigma^2 from
    the warm potentials meets the marginal contract (row error <= 1e-5) well
    before its cap; sampled rows and columns of the plan, summed in FP64 on the
    GPU's potentials, meet it too."""
    laue = gpu_lib
    p = ig.LEARNED
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    q, x = ig.random_grains(p)
    obs = laue.laue_simulate(geom, planes, laue.Grains(q, x), p.sigma_mm, p.distance, p.outlier_frac, p.seed)
    q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, p.seed + 17)
    grains = laue.Grains(q0, x0)
    model = laue.laue_forward_enumerate(geom, planes, grains, True)
    base = laue.ot_defaults(p.sigma_mm, p.distance, model.n)
    c_out, t_b = base.c_out, base.t_b
    s2 = p.sigma_mm ** 2
    ot = laue.ot_params(111.0 * s2, p.distance, c_out, t_b, tol=1e-5, n_max=2000)
    out = laue.laue_em(geom, planes, obs, model, laue.em_params(ot, 111.0 * s2, 3.51 * s2, 4, 4), grains,
                       assign=False)
    assert out["not_converged"] == 0 and out["n_em_iter"] == 16
    eps = 1.11 * s2
    f, g = out["f"], out["g"]
    ot = laue.ot_params(eps, p.distance, c_out, t_b, tol=1e-5, n_max=2000)
    f0, g0, st, rc = laue.laue_sinkhorn(geom, obs, model, ot, f, g, out["f0"], out["g0"])
    print(f"cold stage: {st}")
    assert rc == 0 and st["converged"] and st["err"] <= 1e-5 and st["n_iter"] < 200
    nI = np.diff(obs.block_off)
    nJ = np.diff(model.block_off)
    fc, gc = f.double().cpu().numpy(), g.double().cpu().numpy()
    for b in (int(np.argmax(nI * nJ)), 37, 1):
        Q = laue.laue_plan_block(geom, obs, model, ot, f, g, b).double().cpu().numpy()
        r0, c0 = obs.block_off[b], model.block_off[b]
        q_out = np.exp((fc[r0:r0 + nI[b]] + g0 - c_out) / eps)
        q_unm = np.exp((f0 + gc[c0:c0 + nJ[b]]) / eps)
        assert np.max(np.abs(Q.sum(axis=1) + q_out - 1.0)) < 1.2e-5
        assert np.max(np.abs(Q.sum(axis=0) + q_unm - 1.0)) < 2e-6


def test_network_forward_full_size_sampled(gpu_lib):
    """2^20 candidates through the inference launch (chunks of 65,536 rows):
    sampled rows equal the oracle network's output."""
    laue = gpu_lib
    prm = omlp.init(seed=12)
    prm["b1"] = np.random.default_rng(2).uniform(-0.2, 0.2, 256).astype(np.float32).astype(np.float64)
    net = laue.Mlp(params=laue.Mlp.pack(prm))
    n = 1 << 20
    rng = np.random.default_rng(5)
    feat = rng.uniform(0.0, 1.0, (n, 16)).astype(np.float32)
    prob = laue.laue_mlp_forward(net, torch.tensor(feat, device="cuda")).cpu().numpy()
    rows = np.concatenate([rng.choice(n, 3000, replace=False), [0, 65535, 65536, n - 1]])
    po, _ = omlp.forward(prm, feat[rows].astype(np.float64))
    assert np.max(np.abs(prob[rows] - po)) < 2e-3
    assert np.all(np.isfinite(prob)) and prob.min() > 0.0 and prob.max() < 1.0
