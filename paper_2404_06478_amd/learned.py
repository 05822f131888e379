"""Training the learned proposal on simulated spots, on the GPU.

A training example is one spot-pair candidate of a simulated sample: its 16
features (14 from the pair, 2 cheap-support fractions) and its label (both
spots from one true grain and the orientation within 2 degrees of it;
laue_candidate_labels).  At the densities of interest almost no random pair
comes from one grain, so half of the pairs are drawn among same-grain spots
(laue_pairs_same_grain); their wrong plane hypotheses are negatives as well.
(Labels by the nearest true grain, laue_candidate_labels_nearest, name the
candidates that refinement brings to a grain, but at 1000 grains the features
do not rank them: the network and the support features alone both score
them at chance, the clutter hitting every support probe.)  Every step runs in the
library: simulation, candidates, features, labels, and the network's
forward, backward and Adam kernels, and the batches of each epoch
(laue_mlp_train_epoch draws the seeded example order and gathers them).
"""
from __future__ import annotations

import time

import numpy as np

from . import (Grains, adam_params, laue_candidate_labels, laue_candidate_support, laue_candidates_generate,
               laue_mlp_forward, laue_mlp_train_epoch, laue_pairs_same_grain, laue_simulate)


def sample_examples(geom, planes, truth, sigma_mm, distance, outlier_frac, seed, n_pairs_random,
                    n_pairs_same, support_radius, max_deg=2.0):
    """Features [n, 16] and labels [n] (device FP32) of one simulated sample."""
    import torch
    obs = laue_simulate(geom, planes, truth, sigma_mm, distance, outlier_frac, seed)
    feats, labels = [], []
    a, b = laue_pairs_same_grain(geom, obs, obs.grain, n_pairs_same, seed + 1)
    for pairs, n in ((None, n_pairs_random), ((a, b), n_pairs_same)):
        c = laue_candidates_generate(geom, planes, obs, n, seed + 2, pairs=pairs)
        if c["q"].shape[0] == 0:
            continue
        laue_candidate_support(geom, planes, obs, c, support_radius, planes.n)
        lab, _ = laue_candidate_labels(c, obs.grain, truth, max_deg)
        feats.append(c["feat"])
        labels.append(lab)
    if not feats:
        return torch.zeros((0, 16), device=obs.p1.device), torch.zeros(0, device=obs.p1.device)
    return torch.cat(feats), torch.cat(labels)


def training_set(geom, planes, truths, sigma_mm, distance, outlier_frac, seeds, n_examples,
                 support_radius):
    """At least n_examples examples from the given true grain sets (one sample
    each, in turn, until enough)."""
    import torch
    feats, labels, total, k = [], [], 0, 0
    per = max(1, n_examples // max(len(truths), 1))
    while total < n_examples and k < len(truths):
        # about 15 hypotheses per pair
        n_pairs = max(64, per // 30)
        q, x = truths[k]
        f, l = sample_examples(geom, planes, Grains(q, x), sigma_mm, distance, outlier_frac, seeds[k], n_pairs,
                               n_pairs, support_radius)
        feats.append(f)
        labels.append(l)
        total += f.shape[0]
        k += 1
    return torch.cat(feats)[:n_examples].contiguous(), torch.cat(labels)[:n_examples].contiguous()


def train(net, feat, label, epochs=8, batch=4096, lr=1e-3, seed=0, log=None):
    """Adam on the mean binary cross-entropy, one library epoch call per epoch
    (the library draws each epoch's example order); returns the mean loss per
    epoch."""
    if feat.shape[0] < batch:
        raise ValueError("fewer examples than one batch")
    ap = adam_params(lr=lr)
    out = []
    for ep in range(epochs):
        t0 = time.time()
        out.append(laue_mlp_train_epoch(net, feat, label, batch, seed, ep, ap))
        if log:
            log(f"epoch {ep}: loss {out[-1]:.4f} ({time.time() - t0:.2f} s)")
    return out


def ranking_quality(net, feat, label, top_frac=0.05):
    """Share of positives among the top fraction, recall of positives kept by it,
    and the ROC area (rank statistic)."""
    import torch
    p = laue_mlp_forward(net, feat).double().cpu().numpy()
    y = label.double().cpu().numpy() > 0.5
    n = len(p)
    k = int(np.ceil(top_frac * n))
    order = np.lexsort((np.arange(n), -p))
    top = np.zeros(n, bool)
    top[order[:k]] = True
    n_pos = int(y.sum())
    ranks = np.empty(n)
    ranks[np.argsort(p, kind="stable")] = np.arange(1, n + 1)
    auc = (ranks[y].sum() - n_pos * (n_pos + 1) / 2) / max(n_pos * (n - n_pos), 1)
    return {"n": n, "positives": n_pos, "recall_top": float(y[top].sum() / max(n_pos, 1)),
            "precision_top": float(y[top].mean()) if k else 0.0, "auc": float(auc)}
