"""End-to-end GPU EM against the oracle EM on the tiny configuration."""
import numpy as np
import pytest

import inputgen as ig
from oracle import cost, em as oem, metrics, sinkhorn
from tests import _problems

pytestmark = pytest.mark.gpu


def _run_both(gpu_lib, P, k_gn=2):
    laue = gpu_lib
    p = P.preset
    c_out = cost.c_out(p.sigma_mm, p.distance)
    t_b = sinkhorn.default_tb(len(P.model["m"]))
    eps_list = oem.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    ref = oem.run(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"], P.model, P.q0, P.x0,
                  eps_list, c_out, t_b=t_b, k_gn=k_gn, tol=1e-5, n_max=2000, record=True)
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    grains = laue.Grains(P.q0, P.x0)
    ot = laue.ot_params(p.eps_start, p.distance, c_out, t_b, tol=1e-5, n_max=2000)
    par = laue.em_params(ot, p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage, k_gn=k_gn)
    out = laue.laue_em(geom, planes, obs, model, par, grains)
    return ref, out, grains


def test_em_tiny_matches_oracle(gpu_lib):
    P = _problems.make(ig.TINY)
    ref, out, grains = _run_both(gpu_lib, P)
    qg, xg = grains.numpy()
    mis = np.degrees(metrics.misorientation(qg, ref["q"]))
    assert np.max(mis) < 0.01, mis
    assert np.max(np.linalg.norm(xg - ref["x"], axis=1)) < 0.01
    assert out["n_em_iter"] == 20 and out["not_converged"] == 0
    # both recover the truth to within the noise
    assert np.max(np.degrees(metrics.misorientation(qg, P.q_true))) < 0.1
    # hard assignments agree with the oracle's at its last E-step (the plan of
    # the final potentials at the grains before the last M-step; near-ties
    # aside), and spots not sent to the outlier column go to their true grain
    p = P.preset
    last = ref["stats"][-2]
    C, _, _ = oem.build_costs(P.planes, P.geom, p.distance, P.obs["p12"], P.obs["offsets"],
                              P.model, last["q"], last["x"])
    Pr = sinkhorn.Problem(C, cost.c_out(p.sigma_mm, p.distance), 0.0,
                          cost.c_out(p.sigma_mm, p.distance), ref["t_b"])
    js, _, _ = sinkhorn.hard_assignment(Pr, ref["f"], ref["g"], ref["f0"], ref["g0"], p.eps_end)
    jg = out["j_star"].cpu().numpy()
    assert np.mean(jg == js) > 0.98
    lab = P.obs["grain"]
    gs = out["grain"].cpu().numpy()
    matched = (lab >= 0) & (gs >= 0)
    assert matched.sum() > 0.5 * (lab >= 0).sum()
    assert np.mean(gs[matched] == lab[matched]) > 0.95
    assert out["cost_entries"] > 0


def test_em_noise_free_recovery(gpu_lib):
    P = _problems.make(ig.TINY, sigma=0.0, frac=0.0, seed_shift=3)
    ref, out, grains = _run_both(gpu_lib, P)
    qg, xg = grains.numpy()
    assert np.max(np.degrees(metrics.misorientation(qg, P.q_true))) < 2e-3
    assert np.max(np.linalg.norm(xg - P.x_true, axis=1)) < 2e-3
