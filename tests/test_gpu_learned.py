"""What the trained proposal network gains over the method without it: its
top 5% of the spot-pair candidates of an unseen sample holds several times
more of the good candidates (within 2 degrees of a true grain, both spots
from it) than the 5% that an untrained ranking keeps, and indexing with it
scores far fewer candidates."""
import math

import numpy as np
import pytest
import torch

import inputgen as ig
from paper_2404_06478_amd import learned

pytestmark = pytest.mark.gpu


def test_trained_network_concentrates_good_candidates(gpu_lib):
    laue = gpu_lib
    p = ig.MEDIUM
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    truths = [ig.random_grains(p, seed=p.seed + 2000 + k) for k in range(4)]
    seeds = [p.seed + 2000 + k for k in range(4)]
    feat, lab = learned.training_set(geom, planes, truths, p.sigma_mm, p.distance, p.outlier_frac, seeds,
                                     300_000, support_radius=4.0 * p.sigma_mm)
    assert lab.sum().item() > 1000
    net = laue.Mlp(seed=5)
    untrained = laue.Mlp(seed=5)
    losses = learned.train(net, feat, lab, epochs=6, lr=2e-3)
    assert losses[-1] < losses[0]
    # an unseen sample, random pairs as at inference
    q, x = ig.random_grains(p, seed=p.seed + 2100)
    truth = laue.Grains(q, x)
    obs = laue.laue_simulate(geom, planes, truth, p.sigma_mm, p.distance, p.outlier_frac, p.seed + 2100)
    c = laue.laue_candidates_generate(geom, planes, obs, 12000, 7)
    laue.laue_candidate_support(geom, planes, obs, c, 4.0 * p.sigma_mm, planes.n)
    y, _ = laue.laue_candidate_labels(c, obs.grain, truth, 2.0)
    n_pos = y.sum().item()
    assert n_pos >= 30
    k = math.ceil(0.05 * y.numel())
    kept = {}
    for name, m in (("trained", net), ("untrained", untrained)):
        sel = laue.laue_select_top(laue.laue_mlp_forward(m, c["feat"]), k).long()
        kept[name] = y[sel].sum().item() / n_pos
    print("share of good candidates in the top 5%:", kept)
    assert kept["trained"] >= 0.25
    assert kept["trained"] >= 2.5 * max(kept["untrained"], 0.05)
