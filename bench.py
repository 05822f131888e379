"""Benchmark: Sinkhorn-EM cost-entries/s on one MI355X.

Workload (default "learned-scale"): 1000 BCC grains (a = 2.87 A, planes with
h^2+k^2+l^2 <= 30, band 1-4 A), 60 rotations of 3 deg, two 200 mm detectors at
150 mm, sigma = 1 mm, 70% outliers; detected spots simulated on the GPU; EM
started from the true grains turned by 0.5 deg and moved by 0.5 mm; the
temperature schedule 111 sigma^2 -> 1.11 sigma^2 mm^2 over 5 stages x 4 EM
iterations; Sinkhorn to a relative row-marginal error of 1e-5 (cap 2000).

A step is one EM iteration through the whole path: forward evaluation of the
frozen model spots, the streamed Sinkhorn E-step to tolerance, and two
Gauss-Newton M-step passes.  W warm-up steps run the first W iterations of a
separate run from the same start; the K timed steps are one EM run from the
start (K = 20 is the whole schedule; later steps stay at its last
temperature).  The value is the number of same-block (detected, model) pairs
streamed through cost -> exp -> accumulate in the timed region divided by its
wall time.

One JSON line is printed.  It carries the roofline of the dominant kernel
(the Sinkhorn row/column passes, measured with HIP events inside the library)
and the FP64 oracle timed on a bounded sample on the host CPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

# the library's progress lines (candidates scored, greedy, EM) on stderr, so
# that the index lines' long calls report as they go
os.environ.setdefault("LAUE_LOG", "1")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Roofline of the Sinkhorn passes (ALU-bound; about 1e-1 byte of HBM traffic
# per entry).  Per cost entry the passes issue 16.5 FP32 VALU operations on
# average (17 in the row pass, 16 in the column pass, counted in the compiled
# loop) and 3 transcendentals (sqrt, rcp, exp2).  MI355X: 256 CUs x 4 SIMDs x
# 32 FP32 lanes per clock x 2.4 GHz = 78.6e12 VALU lane-ops/s (the 157.3
# TFLOP/s FP32 vector rate counts an FMA as 2); transcendentals issue at a
# quarter of that rate.  Peak entries/s = 78.6e12 / (16.5 + 4 * 3).
VALU_PER_ENTRY = 16.5
TRANS_PER_ENTRY = 3
VALU_LANE_OPS_PER_S = 256 * 4 * 32 * 2.4e9
PEAK_COMPILED_ENTRIES_PER_S = VALU_LANE_OPS_PER_S / (VALU_PER_ENTRY + 4 * TRANS_PER_ENTRY)
# The line's roofline counts the method's algorithmic work per entry instead
# of the compiled count: about 20 FP32 VALU operations (two differences, the
# cross and dot products, the FMAs of the cost, the potential FMA and the
# accumulation) and 3 transcendentals (square root, reciprocal, exp2).
ALGO_VALU_PER_ENTRY = 20
ALGO_TRANS_PER_ENTRY = 3
PEAK_ENTRIES_PER_S = VALU_LANE_OPS_PER_S / (ALGO_VALU_PER_ENTRY + 4 * ALGO_TRANS_PER_ENTRY)

# HBM bytes of one working row pass (k_row) on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the same
# counters read for a plain 1 GiB device copy (x2.000 and x1.000):
# 78,340 KiB x 2 + 4,456 KiB.  The column pass moves 1.04e8 B.
ROW_PASS_HBM_BYTES = (78_340 * 2.0 + 4_456 * 1.0) * 1024


def build_problem(laue, preset):
    import inputgen as ig
    geom = laue.geometry_from_preset(preset)
    planes = laue.laue_planes_cubic(preset.a, preset.centering, preset.n_max)
    q, x = ig.random_grains(preset)
    obs = laue.laue_simulate(geom, planes, laue.Grains(q, x), preset.sigma_mm, preset.distance,
                             preset.outlier_frac, preset.seed)
    q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, preset.seed + 17)
    grains = laue.Grains(q0, x0)
    model = laue.laue_forward_enumerate(geom, planes, grains, True)
    return geom, planes, obs, model, grains


_POOL = {}


def _oracle_rows(args):
    """Worker of the pooled CPU baseline: the oracle's row half-pass over a
    slice of rows of the shared block (chord cost + log-sum-exp, FP64)."""
    from oracle import cost, sinkhorn
    r0, r1, chunk = args
    d = _POOL
    n_ent = 0
    for r in range(r0, r1, chunk):
        C = cost.chord_cost(d["rows"][r:min(r + chunk, r1)], d["s12"], d["vl"], d["distance"])
        P = sinkhorn.Problem([C], d["c_out"], 0.0, d["c_out"], float(C.shape[1]))
        sinkhorn.row_half(P, d["g"], 0.0, d["eps"])
        n_ent += C.size
    return n_ent


def cpu_baseline(preset, n_rows=10000, chunk=1000, workers=None):
    """The FP64 oracle on a bounded sample: the row half of one Sinkhorn
    iteration (chord cost + log-sum-exp) for detected spots of the largest
    block of one projection, in row chunks; once in this process and once
    split over a pool of worker processes (one per host core, at most 16)."""
    import multiprocessing as mp
    import inputgen as ig
    from oracle import cost, crystal, forward, simulate
    pl = crystal.cubic_planes(preset.a, preset.centering, preset.n_max)
    g = forward.Geometry(1, math.radians(preset.domega_deg), preset.detectors, preset.lam_min,
                         preset.lam_max)
    q, x = ig.random_grains(preset)
    sim = simulate.simulate(pl, q, x, g, preset.sigma_mm, preset.outlier_frac, preset.seed, preset.distance)
    q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, preset.seed + 17)
    mod = forward.enumerate_visible(pl, q0, x0, g)
    b = int(np.argmax(np.bincount(mod["block"], minlength=g.n_blocks)))
    ev = forward.eval_fixed(pl, q0, x0, g, mod["m"], mod["n"], mod["t"], mod["det"])
    sel = mod["block"] == b
    s12, vl = ev["s12"][sel], cost.v_local(g, mod["det"][sel], ev["v"][sel])
    rows = ig.to_f32_exact(sim["p12"][sim["offsets"][b]:sim["offsets"][b + 1]])
    c_out = cost.c_out(preset.sigma_mm, preset.distance)
    _POOL.update(rows=rows, s12=s12, vl=vl, distance=preset.distance, c_out=c_out, g=np.zeros(len(s12)),
                 eps=preset.eps_start)
    n1 = min(n_rows, len(rows))
    t0 = time.perf_counter()
    n_ent = _oracle_rows((0, n1, chunk))
    dt = time.perf_counter() - t0
    single = n_ent / dt
    if workers is None:
        workers = max(1, min(16, os.cpu_count() or 1))
    # each worker takes a slice of the block's rows (the rows repeat if the block is short)
    per = max(chunk, n1 // 2)
    tasks = []
    for w in range(workers):
        r0 = (w * per) % max(len(rows) - per, 1)
        tasks.append((r0, min(r0 + per, len(rows)), chunk))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_rows, [(0, chunk, chunk)] * workers)      # start-up outside the timing
        t0 = time.perf_counter()
        ents = pool.map(_oracle_rows, tasks)
        dtp = time.perf_counter() - t0
    pooled = sum(ents) / dtp
    return {"value": pooled, "unit": "cost-entries/s", "cores": workers, "kind": "oracle",
            "sample": f"row half-pass (chord cost + log-sum-exp, FP64 NumPy) over detected x "
                      f"{len(s12)} model spots of one backscatter block: {workers} processes x {per} rows "
                      f"({sum(ents):.3g} entries, {dtp:.1f} s); one process: {n1} rows ({n_ent:.3g} entries, "
                      f"{dt:.1f} s)",
            "single_process": {"value": single, "cores": 1},
            "host": cpu_host()}


def cpu_host():
    """The host the oracle runs on: CPU model (/proc/cpuinfo), the cores this
    process may use (nproc), os.cpu_count() and the NumPy version."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"cpu_model": model or platform.processor() or platform.machine(), "nproc": nproc,
            "os_cpu_count": os.cpu_count(), "numpy": np.__version__}


def cpu_oracle_runs(n_pairs_tiny=64, n_sample=1):
    """The oracle as written (one process, FP64 NumPy): on the 5-grain
    workload the whole 20-iteration EM and the whole time to index (candidates
    of n_pairs_tiny spot pairs, refinement, scoring, greedy, EM); on the
    100-grain workload the refinement and scoring of n_sample candidates, as
    pairs per second in the library's count (refinement iterations x
    Gauss-Newton steps + 1 passes over the candidate's same-block pairs, plus
    one for a kept candidate), the rate the extrapolations use."""
    import inputgen as ig
    from oracle import candidates, cost, crystal, em, forward, pipeline, simulate, single
    out = {}
    p = ig.TINY
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    g = forward.Geometry.from_preset(p)
    q, x = ig.random_grains(p)
    sim = simulate.simulate(pl, q, x, g, p.sigma_mm, p.outlier_frac, p.seed, p.distance)
    p12 = ig.to_f32_exact(sim["p12"])
    q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, p.seed + 17)
    model = forward.enumerate_visible(pl, q0, x0, g)
    model["offsets"] = forward.block_offsets(model["block"], g.n_blocks)
    sched = em.eps_schedule(p.eps_start, p.eps_end, p.n_stages, p.iters_per_stage)
    c_out = cost.c_out(p.sigma_mm, p.distance)
    t0 = time.perf_counter()
    r = em.run(pl, g, p.distance, p12, sim["offsets"], model, q0, x0, sched, c_out)
    t_em = time.perf_counter() - t0
    t0 = time.perf_counter()
    ix = pipeline.index(pl, g, p.distance, p12, sim["offsets"], p.sigma_mm, c_out, sched, n_pairs_tiny, 1,
                        k_max=2 * p.n_grains)
    t_ix = time.perf_counter() - t0
    out["tiny"] = {"em_iterations": len(sched), "em_s": t_em, "em_iters_per_s": len(sched) / t_em,
                   "sinkhorn_iters": int(sum(s["n_iter"] for s in r["stats"])),
                   "time_to_index_s": t_ix, "pairs": n_pairs_tiny, "candidates": int(len(ix["candidates"]["q"])),
                   "prototypes": int(ix["k"]), "recall": recall(ix["q"], ix["x"], q, x) / len(q),
                   "measured": True}
    pm = ig.MEDIUM
    plm = crystal.cubic_planes(pm.a, pm.centering, pm.n_max)
    gm = forward.Geometry.from_preset(pm)
    qm, xm = ig.random_grains(pm)
    simm = simulate.simulate(plm, qm, xm, gm, pm.sigma_mm, pm.outlier_frac, pm.seed, pm.distance)
    p12m = ig.to_f32_exact(simm["p12"])
    cand = candidates.generate(plm, gm, p12m, simm["offsets"], 2, 1)
    c_outm = cost.c_out(pm.sigma_mm, pm.distance)
    n_blk = np.diff(simm["offsets"])
    pairs, t_sc = 0, 0.0
    for k in range(min(n_sample, len(cand["q"]))):
        t0 = time.perf_counter()
        qq, xx, mod = single.refine(plm, gm, pm.distance, p12m, simm["offsets"], cand["q"][k], np.zeros(3),
                                    pm.sigma_mm, c_outm, k_refine=8, k_gn=1)
        un, nm, rows, vals = single.score(plm, gm, pm.distance, p12m, simm["offsets"], mod, qq, xx, pm.sigma_mm,
                                          c_outm)
        t_sc += time.perf_counter() - t0
        slot = int(np.sum(np.diff(mod["offsets"]) * n_blk))
        pairs += (8 * 1 + 1) * slot + (slot if nm > 0 and un < 0.1 * nm else 0)
    out["medium_scoring_sample"] = {"candidates": min(n_sample, len(cand["q"])), "pairs": pairs, "s": t_sc,
                                    "pairs_per_s": pairs / t_sc if t_sc > 0 else None, "measured": True}
    return out


def cpu_extrapolate(line, base, runs):
    """Oracle time for the GPU lines of this run, extrapolated from the
    oracle's measured rates (labelled so): an EM iteration streams the passes
    the library counted (cost_entries) at the oracle's single-process
    row-pass rate; indexing adds the scoring pairs the library counted at the
    oracle's sampled scoring rate."""
    ent_rate = base["single_process"]["value"]
    pair_rate = runs["medium_scoring_sample"]["pairs_per_s"]
    out = {"note": "extrapolated, one process, from the measured oracle rates (not run)"}
    if line.get("config", {}).get("em_iterations"):
        per_it = line["value"] * line["ms_per_step"] * 1e-3
        out["em_iters_per_s_main_workload"] = ent_rate / per_it
    tti = {}
    for key, v in line.get("time_to_index", {}).items():
        tti[key] = {}
        for mode in ("plain", "learned", "sobol"):
            if mode not in v:
                continue
            x = v[mode]
            em_ent = x.get("em_cost_entries", 0)
            tti[key][mode] = (x["score_pairs"] / pair_rate if pair_rate else None,
                              em_ent / ent_rate)
            tti[key][mode] = {"time_to_index_s": sum(t for t in tti[key][mode] if t is not None),
                              "scoring_s": tti[key][mode][0], "em_s": tti[key][mode][1]}
    out["time_to_index"] = tti
    return out


def misorientation_deg(qa, qb):
    """Smallest rotation angle between cubic orientations, all pairs [na, nb]:
    2 acos of the largest |<dq, s>| over the 24 proper cubic rotations s
    (as quaternions: axis units, (+-e_a +- e_b)/sqrt 2, (+-1,+-1,+-1,+-1)/2)."""
    qa = np.asarray(qa, np.float64)[:, None, :]
    qb = np.asarray(qb, np.float64)[None, :, :]
    w1, x1, y1, z1 = (qa[..., k] for k in range(4))
    w2, x2, y2, z2 = (qb[..., k] for k in range(4))
    # dq = conj(qa) * qb
    d = np.stack([w1 * w2 + x1 * x2 + y1 * y2 + z1 * z2, w1 * x2 - x1 * w2 - y1 * z2 + z1 * y2,
                  w1 * y2 + x1 * z2 - y1 * w2 - z1 * x2, w1 * z2 - x1 * y2 + y1 * x2 - z1 * w2], axis=-1)
    a = -np.sort(-np.abs(d), axis=-1)
    c = np.maximum(a[..., 0], np.maximum((a[..., 0] + a[..., 1]) / math.sqrt(2.0), 0.5 * a.sum(axis=-1)))
    return np.degrees(2.0 * np.arccos(np.clip(c, -1.0, 1.0)))


def recall(q_est, x_est, q_true, x_true, ang_deg=0.25, pos_mm=0.5):
    """True grains matched one-to-one (greedily, by misorientation) by an
    estimate within ang_deg and pos_mm."""
    if len(q_est) == 0:
        return 0
    mis = misorientation_deg(q_true, q_est)
    dist = np.linalg.norm(np.asarray(x_true)[:, None, :] - np.asarray(x_est)[None, :, :], axis=-1)
    ok = (mis <= ang_deg) & (dist <= pos_mm)
    used, n = set(), 0
    for i in np.argsort(np.where(ok, mis, np.inf).min(axis=1)):
        for j in np.argsort(mis[i]):
            if ok[i, j] and j not in used:
                used.add(int(j))
                n += 1
                break
    return n


def bench_batching(laue, n_samples, n_stages, log):
    """64 uneven samples: one batched EM (one launch per pass for all samples)
    against the same samples run one after another."""
    import torch
    import inputgen as ig
    samples = ig.batching_samples(n_samples)
    planes_of, items = {}, []
    for p in samples:
        geom = laue.geometry_from_preset(p)
        key = (p.a, p.centering, p.n_max)
        if key not in planes_of:
            planes_of[key] = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
        planes = planes_of[key]
        q, x = ig.random_grains(p)
        obs = laue.laue_simulate(geom, planes, laue.Grains(q, x), p.sigma_mm, p.distance, p.outlier_frac, p.seed)
        q0, x0 = ig.perturb_grains(q, x, 0.5, 0.5, p.seed + 17)
        model = laue.laue_forward_enumerate(geom, planes, laue.Grains(q0, x0), True)
        base = laue.ot_defaults(p.sigma_mm, p.distance, model.n)
        ot = laue.ot_params(p.eps_start, p.distance, base.c_out, base.t_b)
        par = laue.em_params(ot, p.eps_start, p.eps_end, n_stages, 1)
        items.append((geom, planes, obs, model, par, (q0, x0), p))
    log(f"batching: {n_samples} samples, {sum(it[2].n for it in items)} detected and "
        f"{sum(it[3].n for it in items)} model spots in all")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq, seq_entries, seq_pass_ms, seq_pass_entries = [], 0, 0.0, 0
    for geom, planes, obs, model, par, (q0, x0), _ in items:
        gr = laue.Grains(q0, x0)
        o = laue.laue_em(geom, planes, obs, model, par, gr, assign=False)
        seq.append(gr)
        seq_entries += o["cost_entries"]
        seq_pass_ms += o["sinkhorn_ms"] + o["mstep_ms"]
        seq_pass_entries += o["sinkhorn_entries"] + o["mstep_entries"]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log(f"batching: sequential {t_seq:.2f} s")
    grains = [laue.Grains(*it[5]) for it in items]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, outs = laue.laue_em_batched([it[0] for it in items], [it[1] for it in items], [it[2] for it in items],
                                    [it[3] for it in items], [it[4] for it in items], grains, assign=False)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    log(f"batching: batched {t_b:.2f} s")
    b_entries = sum(o["cost_entries"] for o in outs)
    # pass time (HIP events around the Sinkhorn and M-step passes, the batch's
    # totals in every entry of a batched call) and the entries it covers
    b_pass_ms = outs[0]["sinkhorn_ms"] + outs[0]["mstep_ms"]
    b_pass_entries = sum(o["sinkhorn_entries"] + o["mstep_entries"] for o in outs)
    same = all(torch.equal(a.q, b.q) and torch.equal(a.x, b.x) for a, b in zip(seq, grains))
    return {"samples": n_samples, "em_iterations": n_stages,
            "grains": [int(it[6].n_grains) for it in items][:8] + ["..."],
            "sequential_s": t_seq, "batched_s": t_b, "speedup": t_seq / t_b,
            "sequential_entries_per_s": seq_entries / t_seq, "batched_entries_per_s": b_entries / t_b,
            "batched_em_iters_per_s": n_samples * n_stages / t_b,
            "passes": {"sequential_ms": seq_pass_ms, "batched_ms": b_pass_ms,
                       "sequential_share_of_wall": seq_pass_ms * 1e-3 / t_seq,
                       "batched_share_of_wall": b_pass_ms * 1e-3 / t_b,
                       "sequential_entries_per_s": seq_pass_entries / max(seq_pass_ms * 1e-3, 1e-12),
                       "batched_entries_per_s": b_pass_entries / max(b_pass_ms * 1e-3, 1e-12)},
            "launch_used": outs[0]["launch_used"], "identical_to_sequential": bool(same)}


def recipe_params(laue, p, recipe, n_obs, rho=0):
    """Refinement and EM parameters of an index line.  "stages": the
    refinement 30 -> 1.11 sigma^2 in 8 iterations and the EM's 5 x 4 stage
    schedule 111 -> 1.11 sigma^2.  "paper": the paper's annealing (Sec. 5.1,
    Sec. 7, App. D): the refinement cools by 0.97 per iteration from 30 sigma^2
    to 2 sigma^2 (90 iterations, one Gauss-Newton step each), the EM cools by
    0.97 per iteration from the data-tied first temperature (the farthest of 32
    neighbours, computed by the library) to 2 sigma^2 (the paper's temperature
    1), then at most 20 more iterations with the plan-change stop.  rho > 0:
    the EM's E-step keeps each detected spot's rho nearest model spots (the
    paper's sparse assignment, Sec. 5.2)."""
    s2 = p.sigma_mm ** 2
    c_out = laue.c_out_3sigma(p.sigma_mm, p.distance)
    if recipe == "stages":
        return None, None
    score = laue.score_params(p.sigma_mm, p.distance, c_out, k_refine=90, k_gn=1, eps_start=30.0 * s2,
                              eps_cool=0.97)
    ot = laue.ot_params(1.0, p.distance, c_out, 0.0, rho=rho)
    em = laue.em_params(ot, 0.0, 2.0 * s2, 1, 1, eps_cool=0.97, final_iters=20,
                        zeta_tol=ZETA_TOL_PER_ROOT_SPOT * math.sqrt(max(n_obs, 1)), sigma_mm=p.sigma_mm)
    return score, em


# Plan-change stop of the paper's EM recipe: ||Q^{k+1} - Q^k||_F <= this times
# sqrt(detected spots), i.e. an RMS change per detected spot's row of 1e-3.
ZETA_TOL_PER_ROOT_SPOT = 1e-3


def bench_index(laue, workload, n_pairs, learned_pairs, log, sobol_points=0, recipe="stages", max_candidates=None,
                plain_max=None, train_examples=1_000_000, spot_per_candidate=None, rho=0):
    """Time to index from device-resident spots (laue_index): plain exhaustive
    scoring of the candidates of n_pairs spot pairs, against (learned_pairs >
    0) the learned proposal scoring the top 5% of the candidates of
    learned_pairs pairs, with a network trained here on 10^6 simulated
    examples, and (sobol_points > 0)
    the paper's Sobol-grid starts over the cubic fundamental zone and the
    sample box.  max_candidates caps the candidates of both forms (the first
    ones); plain_max caps the plain form's alone; spot_per_candidate sizes the
    Sobol form's SPOT matrix (entries per start) where the default guess would
    not fit."""
    import torch
    import inputgen as ig
    from paper_2404_06478_amd import learned
    p = ig.PRESETS[workload]
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    radius = 4.0 * p.sigma_mm
    net, training = None, None
    if learned_pairs:
        truths = [ig.random_grains(p, seed=p.seed + 1000 + k) for k in range(10)]
        seeds = [p.seed + 1000 + k for k in range(10)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        feat, lab = learned.training_set(geom, planes, truths, p.sigma_mm, p.distance, p.outlier_frac, seeds,
                                         train_examples, support_radius=radius)
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        net = laue.Mlp(seed=3)
        t0 = time.perf_counter()
        losses = learned.train(net, feat, lab, epochs=10, lr=2e-3)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        log(f"index: training set {feat.shape[0]} examples in {t_data:.1f} s, 10 epochs in {t_train:.1f} s")
        training = {"examples": int(feat.shape[0]), "positives": int(lab.sum().item()), "data_s": t_data,
                    "train_s": t_train, "epochs": 10, "final_loss": losses[-1]}
    q, x = ig.random_grains(p)
    obs = laue.laue_simulate(geom, planes, laue.Grains(q, x), p.sigma_mm, p.distance, p.outlier_frac, p.seed)
    out = {"workload": workload, "grains": p.n_grains, "detected_spots": obs.n, "recipe": recipe,
           "training": training, "rho": rho}
    # the sparse E-step (rho) for the Sobol form's EM only: its prototypes give
    # hundreds of model spots per block; the pair forms' few dozen
    # prototypes leave fewer model spots per block than rho, where choosing
    # neighbours at every E-step costs more than the dense passes it saves
    score, em = recipe_params(laue, p, recipe, obs.n)
    em_sobol = recipe_params(laue, p, recipe, obs.n, rho)[1]
    modes = [("plain", n_pairs)] + ([("learned", learned_pairs)] if learned_pairs else []) + \
        ([("sobol", sobol_points)] if sobol_points else [])
    for mode, pairs in modes:
        mc = max_candidates if mode != "plain" or plain_max is None else plain_max
        if mode == "sobol":
            # dense samples keep nearly every start, each with thousands of
            # SPOT entries: size the SPOT matrix for the starts (64-bit offsets)
            cap = 8000 * pairs if obs.n * pairs > 1e11 else None
            cap = spot_per_candidate * pairs if spot_per_candidate else cap
            par = laue.index_params(p, "sobol", max_candidates=pairs, n_obs=obs.n, n_planes=planes.n, lbar_cap=cap,
                                    score=score, em=em_sobol)
        else:
            n_sc = mc if mc is not None else 64 * pairs
            n_sc = int(math.ceil(0.05 * n_sc)) if mode == "learned" else n_sc
            # dense clutter keeps nearly every candidate, each with an entry for
            # most detected spots within reach: size the SPOT matrix for it
            cap = (8000 if p.n_grains <= 1000 else 32000) * n_sc if obs.n * n_sc > 1e11 else None
            par = laue.index_params(p, mode, n_pairs=pairs, seed=1, mlp=net if mode == "learned" else None,
                                    support_radius=radius, n_obs=obs.n, n_planes=planes.n, max_candidates=mc,
                                    lbar_cap=cap, score=score, em=em)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g, st, _ = laue.laue_index(geom, planes, obs, par, assign=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        qg, xg = g.numpy()
        r = recall(qg[:g.n], xg[:g.n], q, x)
        out[mode] = {("sobol_points" if mode == "sobol" else "pairs"): pairs, "candidates": st["n_candidates"],
                     "candidates_found": st["n_candidates_found"], "scored": st["n_scored"],
                     "em_iterations": st["em"]["n_em_iter"], "em_sinkhorn_capped": st["em"]["not_converged"],
                     "em_cost_entries": st["em"]["cost_entries"],
                     "em_zeta": st["em"]["zeta"], "likelihood": st["em"]["objective"]["sem_objective"],
                     "spot_entries": st["lbar_entries"], "prototypes": st["n_prototypes"], "recall": r / len(q),
                     "time_s": wall,
                     "score_pairs": st["score_pairs"], "score_pairs_evaluated": st["score_pairs_evaluated"],
                     "score_pairs_refine": st["score_pairs_refine"],
                     "score_pairs_per_s": st["score_pairs"] / max(st["ms_score"] * 1e-3, 1e-12),
                     "stage_ms": {k: st[k] for k in ("ms_candidates", "ms_proposal", "ms_score", "ms_greedy",
                                                     "ms_em")}}
        log(f"index: {mode}: {pairs} {'points' if mode == 'sobol' else 'pairs'}, {st['n_scored']} scored, "
            f"recall {r}/{len(q)}, {wall:.2f} s (the refinement and scoring passes evaluated "
            f"{st['score_pairs_evaluated'] / max(st['score_pairs'], 1):.4f} of their pairs)")
    return out


def _per_grain(q, x, qg, xg):
    mis = np.diag(misorientation_deg(q, qg))
    dx = np.linalg.norm(np.asarray(x) - np.asarray(xg), axis=1)
    return {"within_0.25deg_0.5mm": int(np.sum((mis <= 0.25) & (dx <= 0.5))),
            "median_deg": float(np.median(mis)), "median_mm": float(np.median(dx))}


def _geometric(e0, e1, n):
    return [e0 * (e1 / e0) ** (k / max(n - 1, 1)) for k in range(n)]


def bench_index_limits(laue, preset, log, n_random=9000):
    """Where indexing at a spot density holds and where it breaks, on one
    simulated sample: (i) the multi-grain EM started from the true grains, at
    the schedule's first temperature (111 sigma^2, four iterations) and on a
    cold schedule (3.51 -> 1.11 sigma^2, eight iterations); (ii) the EM from
    the true grains turned by 0.5 deg and moved by 0.5 mm (7.9 -> 1.11 sigma^2,
    twenty iterations); (iii) single-grain refinement and SPOT selection of
    candidates made of those turned grains mixed with n_random random grains.
    A grain counts when it ends within 0.25 deg and 0.5 mm of its own true
    grain."""
    import torch
    import inputgen as ig
    geom = laue.geometry_from_preset(preset)
    planes = laue.laue_planes_cubic(preset.a, preset.centering, preset.n_max)
    q, x = ig.random_grains(preset)
    obs = laue.laue_simulate(geom, planes, laue.Grains(q, x), preset.sigma_mm, preset.distance,
                             preset.outlier_frac, preset.seed)
    s2 = preset.sigma_mm ** 2
    c_out = _c_out(preset)
    qt, xt = ig.perturb_grains(q, x, 0.5, 0.5, preset.seed + 17)
    dev = torch.device("cuda", 0)
    out = {"workload": preset.name, "grains": len(q), "detected_spots": obs.n}

    def em(q0, x0, sched):
        grains = laue.Grains(q0, x0)
        model = laue.laue_forward_enumerate(geom, planes, grains, True)
        t_b = laue.ot_defaults(preset.sigma_mm, preset.distance, model.n).t_b
        f = torch.zeros(obs.n, dtype=torch.float32, device=dev)
        g = torch.zeros(model.n, dtype=torch.float32, device=dev)
        f0 = g0 = 0.0
        for eps in sched:
            ot = laue.ot_params(eps, preset.distance, c_out, t_b, tol=1e-5, n_max=2000)
            o = laue.laue_em(geom, planes, obs, model, laue.em_params(ot, eps, eps, 1, 1, k_gn=2), grains, f, g,
                             f0, g0, assign=False)
            f0, g0 = o["f0"], o["g0"]
        qg, xg = grains.numpy()
        return dict(_per_grain(q, x, qg, xg), eps_mm2=[round(sched[0], 4), round(sched[-1], 4)],
                    iterations=len(sched))

    out["em_hot_from_truth"] = em(q, x, [111.0 * s2] * 4)
    out["em_cold_from_truth"] = em(q, x, _geometric(3.51 * s2, 1.11 * s2, 8))
    out["em_from_turned"] = em(qt, xt, _geometric(7.9 * s2, 1.11 * s2, 20))
    log(f"index limits {preset.name}: EM from truth hot {out['em_hot_from_truth']['within_0.25deg_0.5mm']}, "
        f"cold {out['em_cold_from_truth']['within_0.25deg_0.5mm']}, from 0.5 deg "
        f"{out['em_from_turned']['within_0.25deg_0.5mm']} of {len(q)}")
    qr, xr = ig.random_grains(preset, n=n_random, seed=preset.seed + 4242)
    ng = len(q)
    cand = laue.Grains(np.concatenate([qt, qr]), np.concatenate([xt, xr]))
    phi = -c_out / (2.0 * s2)
    r = laue.laue_score_candidates(geom, planes, obs, cand, laue.score_params(preset.sigma_mm, preset.distance,
                                                                              c_out),
                                   lbar_cap=min((1 << 31) - 1, 12_000 * (ng + n_random)))
    rq, rx = cand.numpy()
    refined = _per_grain(q, x, rq[:ng], rx[:ng])
    ok = (np.diag(misorientation_deg(q, rq[:ng])) <= 0.25) & (np.linalg.norm(x - rx[:ng], axis=1) <= 0.5)
    keep = r["keep"].cpu().numpy().astype(bool)
    off = r["lbar_off"].cpu().numpy()
    cs = np.concatenate([[0.0], np.cumsum(r["lbar_val"].cpu().numpy().astype(np.float64) - phi)])
    col = cs[off[1:]] - cs[off[:-1]]
    picks, gains = laue.laue_spot_greedy(r["lbar_off"], r["lbar_row"], r["lbar_val"], ng + n_random, obs.n, phi, ng)
    pk = picks.cpu().numpy()
    gn = gains.cpu().numpy()
    drop = gn - np.append(gn[1:], 0.0)
    out["selection"] = {
        "candidates": {"turned_true": ng, "random": n_random}, "spot_entries": int(r["lbar_n"]),
        "refined_turned": refined, "kept_turned": float(keep[:ng].mean()), "kept_random": float(keep[ng:].mean()),
        "column_sum_turned_median": float(np.median(col[:ng])),
        "column_sum_random_median": float(np.median(col[ng:])),
        "column_sum_random_p99": float(np.percentile(col[ng:], 99)),
        "first_picks": int(len(pk)), "picks_turned": int(np.sum(pk < ng)),
        "picks_turned_within": int(np.sum(ok[pk[pk < ng]])), "k_star": int(np.argmax(drop)) + 1 if len(gn) else 0}
    sel = out["selection"]
    log(f"index limits {preset.name}: refined {refined['within_0.25deg_0.5mm']}/{ng}, kept turned "
        f"{sel['kept_turned']:.2f} random {sel['kept_random']:.2f}, first {len(pk)} picks: {sel['picks_turned']} "
        f"turned ({sel['picks_turned_within']} within), k* {sel['k_star']}")
    return out


def _em_schedule(preset):
    return [preset.eps_start * (preset.eps_end / preset.eps_start) ** (s / (preset.n_stages - 1))
            for s in range(preset.n_stages) for _ in range(preset.iters_per_stage)]


def _c_out(preset):
    import paper_2404_06478_amd as laue
    return laue.c_out_3sigma(preset.sigma_mm, preset.distance)


def _em_iterations(laue, preset, ks, log, label, em_kw=None, **ot_kw):
    """EM iterations ks of the schedule from the same start (fresh problem,
    zero potentials), each one laue_em call of one iteration; returns the
    per-iteration stats summary and the final grains."""
    import torch
    eps_list = _em_schedule(preset)
    geom, planes, obs, model, grains = build_problem(laue, preset)
    t_b = laue.ot_defaults(preset.sigma_mm, preset.distance, model.n).t_b
    dev = torch.device("cuda", 0)
    f = torch.zeros(obs.n, dtype=torch.float32, device=dev)
    g = torch.zeros(model.n, dtype=torch.float32, device=dev)
    f0 = g0 = 0.0
    stats = []
    extra = {}
    if ot_kw.get("rho"):
        nbr, cst, _ = laue.laue_sparse_neighbors(
            geom, obs, model, laue.ot_params(1.0, preset.distance, _c_out(preset), 1.0, rho=ot_kw["rho"]))
        far = cst[:, -1].double().cpu().numpy()
        far = far[np.isfinite(far)]
        extra["eps_init_mm2"] = float(np.median(far) / math.log(100.0)) if len(far) else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in ks:
        eps = eps_list[k % len(eps_list)]
        ot = laue.ot_params(eps, preset.distance, _c_out(preset), t_b, tol=1e-5, n_max=2000, **ot_kw)
        par = laue.em_params(ot, eps, eps, 1, 1, **(em_kw or {"k_gn": 2}))
        o = laue.laue_em(geom, planes, obs, model, par, grains, f, g, f0, g0, assign=False)
        if not ot_kw.get("unbalanced_kl") and not ot_kw.get("partial_frac"):
            f0, g0 = o["f0"], o["g0"]
        stats.append(o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    qg, xg = grains.numpy()
    sk_ms = sum(s["sinkhorn_ms"] for s in stats)
    summ = {"ms_per_em_iteration": dt * 1e3 / len(ks),
            "sinkhorn_iters": int(sum(s["sinkhorn_iters"] for s in stats)),
            "not_converged": int(sum(s["not_converged"] for s in stats)),
            "pass_pairs": int(sum(s["sinkhorn_entries"] for s in stats)),
            "pass_pairs_per_s": sum(s["sinkhorn_entries"] for s in stats) / max(sk_ms * 1e-3, 1e-12),
            "sinkhorn_ms": sk_ms, "mstep_ms": sum(s["mstep_ms"] for s in stats)}
    log(f"{label}: {dt * 1e3 / len(ks):.1f} ms per EM iteration")
    return summ, qg, xg, extra


def _deviation(a, b):
    mis = np.diag(misorientation_deg(a[0], b[0]))
    dx = np.linalg.norm(a[1] - b[1], axis=1)
    return {"max_misorientation_deg": float(mis.max()), "median_misorientation_deg": float(np.median(mis)),
            "max_position_mm": float(dx.max()), "median_position_mm": float(np.median(dx))}


def bench_sparse(laue, preset, rho, n_iter, log, first_iter=8):
    """The same EM iterations from the same start, dense and with the sparse
    assignment (each detected spot keeps its rho nearest model spots, sets
    rebuilt before every Sinkhorn): time per iteration, the sparse passes'
    pairs/s, and how far the sparse grains end from the dense ones.  The
    iterations start at first_iter of the schedule (stage 2, eps = 11.1
    sigma^2): the paper starts a sparse EM at a temperature tied to the
    farthest kept neighbour, reported here as median c_(rho) / ln 100."""
    import inputgen as ig
    q, x = ig.random_grains(preset)
    eps_list = _em_schedule(preset)
    ks = list(range(first_iter, first_iter + n_iter))
    out = {"rho": rho, "em_iterations": [first_iter, first_iter + n_iter],
           "eps_mm2": sorted({round(eps_list[k % len(eps_list)], 4) for k in ks}, reverse=True)}
    res = {}
    for r in (0, rho):
        key = "dense" if r == 0 else "sparse"
        summ, qg, xg, extra = _em_iterations(laue, preset, ks, log, f"sparse: rho={r}", rho=r)
        summ["recall_0.25deg_0.5mm"] = recall(qg, xg, q, x) / len(q)
        out[key] = summ
        out.update(extra)
        res[r] = (qg, xg)
    out["speedup"] = out["dense"]["ms_per_em_iteration"] / out["sparse"]["ms_per_em_iteration"]
    out["sparse_vs_dense"] = _deviation(res[rho], res[0])
    return out


def bench_outlier_models(laue, preset, kls, fracs, n_iter, log, first_iter=0):
    """The same EM iterations from the same start with the paper's outlier
    row and column, with unbalanced OT at each (kappa, lambda) of kls (units
    of 2 sigma^2, the paper's log-likelihood units) and with partial OT at
    each transported fraction of fracs: time per iteration, the passes'
    entries/s (same streamed kernels, other epilogue), Sinkhorn iterations,
    recall, and how far the grains end from those of the paper's model.  Run
    on a workload where the paper's model recovers the grains (100 grains,
    30% outliers), so that recall compares the outlier treatments."""
    import inputgen as ig
    q, x = ig.random_grains(preset)
    eps_list = _em_schedule(preset)
    ks = list(range(first_iter, first_iter + n_iter))
    s2 = 2.0 * preset.sigma_mm ** 2
    out = {"em_iterations": [first_iter, first_iter + n_iter],
           "eps_mm2": sorted({round(eps_list[k % len(eps_list)], 4) for k in ks}, reverse=True)}
    summ, qb, xb, _ = _em_iterations(laue, preset, ks, log, "unbalanced: outlier bins")
    summ["recall_0.25deg_0.5mm"] = recall(qb, xb, q, x) / len(q)
    out["outlier_bins"] = summ
    out["unbalanced"] = []
    for kl in kls:
        summ, qg, xg, _ = _em_iterations(laue, preset, ks, log, f"unbalanced: kappa, lambda = {kl}",
                                         unbalanced_kl=(kl[0] * s2, kl[1] * s2))
        summ["kappa_lambda_2sigma2"] = list(kl)
        summ["kappa_lambda_mm2"] = [kl[0] * s2, kl[1] * s2]
        summ["recall_0.25deg_0.5mm"] = recall(qg, xg, q, x) / len(q)
        summ["vs_outlier_bins"] = _deviation((qg, xg), (qb, xb))
        out["unbalanced"].append(summ)
    out["partial"] = []
    for frac in fracs:
        summ, qg, xg, _ = _em_iterations(laue, preset, ks, log, f"partial: m_OT = {frac}", partial_frac=frac)
        summ["m_frac"] = frac
        summ["recall_0.25deg_0.5mm"] = recall(qg, xg, q, x) / len(q)
        summ["vs_outlier_bins"] = _deviation((qg, xg), (qb, xb))
        out["partial"].append(summ)
    return out


def bench_mstep_methods(laue, preset, quality_preset, n_iter, log, first_iter=2):
    """The paper's coordinate-descent M-step (one or two sweeps of
    LauePosNewton, 3 steps, then LaueRotMM) against the joint Gauss-Newton
    M-step (2 steps):
    time per EM iteration and in the M-step on preset (EM iterations
    first_iter.. of the schedule, the throughput metric's iterations), and
    recall over the whole schedule on quality_preset."""
    import inputgen as ig
    cd = {"mstep": "paper", "k_newton": 3, "k_mm": 500, "tol_x": 1e-6, "tol_r": 1e-12}
    kws = {"gauss_newton": {"k_gn": 2}, "paper": dict(cd, k_gn=1), "paper_2_sweeps": dict(cd, k_gn=2)}
    out = {"em_iterations": [first_iter, first_iter + n_iter], "settings": kws}
    res = {}
    for key, kw in kws.items():
        summ, qg, xg, _ = _em_iterations(laue, preset, list(range(first_iter, first_iter + n_iter)), log,
                                         f"mstep: {key}", em_kw=kw)
        out[key] = summ
        res[key] = (qg, xg)
    out["paper_vs_gauss_newton"] = _deviation(res["paper"], res["gauss_newton"])
    out["paper_2_sweeps_vs_gauss_newton"] = _deviation(res["paper_2_sweeps"], res["gauss_newton"])
    q, x = ig.random_grains(quality_preset)
    ks = list(range(len(_em_schedule(quality_preset))))
    out["quality"] = {"workload": quality_preset.name, "em_iterations": [0, len(ks)]}
    for key, kw in kws.items():
        summ, qg, xg, _ = _em_iterations(laue, quality_preset, ks, log, f"mstep quality: {key}", em_kw=kw)
        out["quality"][key] = {"ms_per_em_iteration": summ["ms_per_em_iteration"], "mstep_ms": summ["mstep_ms"],
                               "recall_0.25deg_0.5mm": recall(qg, xg, q, x) / len(q)}
    return out


def bench_forward(laue, n_grains, log):
    """Forward model at candidate scale: enumerate the visible reflections of
    n_grains random grains (learned-scale scan and lattice), then time the
    frozen-list evaluation (ids in: 12 B; s1, s2, vn, v1, v2, lambda out:
    24 B per model spot) against the 8 TB/s HBM peak."""
    import torch
    import inputgen as ig
    p = ig.LEARNED
    geom = laue.geometry_from_preset(p)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    q, x = ig.random_grains(p, n=n_grains, seed=p.seed + 7)
    grains = laue.Grains(q, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    model = laue.laue_forward_enumerate(geom, planes, grains, True)
    torch.cuda.synchronize()
    t_enum = time.perf_counter() - t0
    laue.laue_forward_eval(geom, planes, grains, model)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 10
    ev[0].record()
    for _ in range(reps):
        laue.laue_forward_eval(geom, planes, grains, model)
    ev[1].record()
    torch.cuda.synchronize()
    t_eval = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
    nbytes = 36.0 * model.n
    log(f"forward: {n_grains} grains, {model.n} model spots, enumerate {t_enum * 1e3:.1f} ms, "
        f"eval {t_eval * 1e3:.3f} ms")
    triples = n_grains * p.n_rot * planes.n
    return {"grains": n_grains, "model_spots": model.n, "triples": triples,
            "enumerate_s": t_enum, "enumerate_triples_per_s": triples / t_enum,
            "eval_ms": t_eval * 1e3, "eval_bytes": nbytes, "eval_GBps": nbytes / t_eval / 1e9,
            "eval_hbm_frac": nbytes / t_eval / 8e12}


# Index lines of the default run: the 100-grain workload (stage schedule);
# the 1000-grain target workload as its configuration states it (2^20
# spot-pair candidates: the network ranks them and the top 5% are scored,
# against plain scoring of all 2^20), on the stage schedule; the same sample
# at the paper's fiducial noise with the paper's annealing recipe, the same
# 100 grains; 1000 grains at 70% outliers (2^20 candidates both ways); 1000
# grains at the paper's fiducial noise with the paper's recipe (plain scoring
# of 2048 pairs' candidates, about the recall the learned form reaches from
# the top 5% of 2^20, and 3,000,000 Sobol-grid starts, whose EM keeps each
# detected spot's 32 nearest model spots as the paper's does); the 2000-grain stress
# workload (the network ranks 2^20 candidates and scores the top 5%; plain
# scoring of the first 2^16).
DEFAULT_INDEX_LINES = ("medium,pairs=8192,sobol=200000;"
                       "learned,pairs=32768,lpairs=32768,cand=1048576;"
                       "learned_fiducial,pairs=2048,lpairs=24576,cand=1048576,sobol=3000000,spot=64,recipe=paper,rho=32;"
                       "stress,pairs=32768,lpairs=32768,cand=1048576,pcand=65536")


def parse_index_line(item):
    parts = [x.strip() for x in item.split(",") if x.strip()]
    o = {"pairs": 4096, "lpairs": None, "sobol": 0, "recipe": "stages", "cand": None, "pcand": None,
         "examples": 1_000_000, "spot": None, "rho": 0}
    for kv in parts[1:]:
        k, v = kv.split("=")
        if k not in o and k != "name":
            raise ValueError(f"unknown index-line option {k}")
        o[k] = v if k in ("recipe", "name") else int(v)
    if o["lpairs"] is None:
        o["lpairs"] = 8 * o["pairs"]
    if o["recipe"] not in ("stages", "paper"):
        raise ValueError("recipe must be stages or paper")
    if o["rho"] and o["recipe"] != "paper":
        raise ValueError("rho applies to the paper recipe's EM")
    return parts[0], o


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="EM iterations timed: one run from the start "
                    "(20 = the whole schedule; more continue at its last temperature)")
    ap.add_argument("--warmup", type=int, default=2, help="iterations of a separate untimed run first")
    ap.add_argument("--workload", default="learned", choices=["learned", "medium", "stress"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--no-index", action="store_true")
    ap.add_argument("--no-forward", action="store_true")
    ap.add_argument("--forward-grains", type=int, default=65536)
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--sparse-rho", type=int, default=32)
    ap.add_argument("--sparse-iters", type=int, default=8)
    ap.add_argument("--no-unbalanced", action="store_true")
    ap.add_argument("--unbalanced-kl", default="0.01,0.01;0.1,0.1;1,1",
                    help="kappa,lambda pairs (';'-separated) of unbalanced OT in units of 2 sigma^2 "
                         "(the paper's log-likelihood units)")
    ap.add_argument("--unbalanced-iters", type=int, default=20)
    ap.add_argument("--partial-fracs", default="0.5,0.7,0.9", help="m_OT values of partial OT")
    ap.add_argument("--unbalanced-workload", default="medium", choices=["medium", "learned", "stress"])
    ap.add_argument("--no-mstep-methods", action="store_true")
    ap.add_argument("--batch-samples", type=int, default=64)
    ap.add_argument("--index-workloads", default=DEFAULT_INDEX_LINES,
                    help="';'-separated index lines, each 'workload' followed by ',key=value' options: pairs "
                         "(plain form's spot pairs), lpairs (learned form's, default 8 x pairs; 0: no learned form), "
                         "sobol (Sobol points, "
                         "0: none), recipe (stages or paper), cand (candidate cap of both forms), pcand (plain "
                         "form's cap), examples (training examples), spot (SPOT entries per Sobol start), rho "
                         "(the paper recipe's sparse E-step in the Sobol form's EM: nearest model spots kept per detected "
                         "spot; 0: dense)")
    ap.add_argument("--index-limits", default="",
                    help="workloads of the EM-from-truth and selection diagnostics ('' to skip)")
    ap.add_argument("--tile", type=int, default=0, choices=[0, 1, 2],
                    help="Sinkhorn tile shape: 1 or 2 spots per lane, 0 tuned per call")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device three times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)
    import torch
    import inputgen as ig
    import paper_2404_06478_amd as laue
    laue.require_native()
    torch.cuda.set_device(0)
    preset = ig.PRESETS[args.workload]
    geom, planes, obs, model, grains = build_problem(laue, preset)
    q_start, x_start = grains.numpy()
    # the outlier row and column of Sec. 7 (3-sigma outlier cost, T_b = ceil(0.4 |J|))
    base = laue.ot_defaults(preset.sigma_mm, preset.distance, model.n)
    c_out, t_b = base.c_out, base.t_b
    eps_list = _em_schedule(preset)
    n_sched = len(eps_list)
    dev = torch.device("cuda", 0)

    def fresh():
        return (laue.Grains(q_start, x_start), torch.zeros(obs.n, dtype=torch.float32, device=dev),
                torch.zeros(model.n, dtype=torch.float32, device=dev), {"f0": 0.0, "g0": 0.0})

    def step(k, state):
        # iteration k of one EM run from the start: the schedule's temperature,
        # then (steps beyond it) its last temperature
        gr, f, g, pot = state
        eps = eps_list[min(k, n_sched - 1)]
        ot = laue.ot_params(eps, preset.distance, c_out, t_b, tol=1e-5, n_max=2000)
        par = laue.em_params(ot, eps, eps, 1, 1, k_gn=2, tile=args.tile)
        out = laue.laue_em(geom, planes, obs, model, par, gr, f, g, pot["f0"], pot["g0"], assign=False)
        pot["f0"], pot["g0"] = out["f0"], out["g0"]
        return out

    print(f"bench: {args.workload}: {obs.n} detected, {model.n} model spots, "
          f"{int(np.sum(np.diff(obs.block_off) * np.diff(model.block_off)))} entries per pass",
          file=sys.stderr, flush=True)
    # warm-up: the first W iterations of a separate run from the same start
    warm = fresh()
    for k in range(args.warmup):
        o = step(k, warm)
        print(f"bench: warm-up step {k}: {o['sinkhorn_iters']} Sinkhorn iterations", file=sys.stderr, flush=True)
    del warm
    # timed: K iterations of one EM run from the start (no wrap of the schedule)
    state = fresh()
    torch.cuda.synchronize()
    stats, step_s = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        stats.append(step(k, state))
        step_s.append(time.perf_counter() - ts)
        print(f"bench: step {k}: eps {eps_list[min(k, n_sched - 1)]:.3g}, {stats[-1]['sinkhorn_iters']} Sinkhorn "
              f"iterations (err {stats[-1]['last_err']:.2e}), {step_s[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    entries = sum(s["cost_entries"] for s in stats)
    sk_ms = sum(s["sinkhorn_ms"] for s in stats)
    sk_ent = sum(s["sinkhorn_entries"] for s in stats)
    sk_pass = sum(s["sinkhorn_passes"] for s in stats)
    achieved = sk_ent / (sk_ms * 1e-3)
    blk_i = np.diff(obs.block_off)
    blk_j = np.diff(model.block_off)
    qf, xf = state[0].numpy()
    q_true, x_true = ig.random_grains(preset)
    stages = []
    for k, s in enumerate(stats):
        e = round(eps_list[min(k, n_sched - 1)], 6)
        if not stages or stages[-1]["eps_mm2"] != e:
            stages.append({"eps_mm2": e, "em_iterations": 0, "sinkhorn_iters": 0, "ms": 0.0, "capped": 0})
        st = stages[-1]
        st["em_iterations"] += 1
        st["sinkhorn_iters"] += int(s["sinkhorn_iters"])
        st["ms"] += step_s[k] * 1e3
        st["capped"] += int(s["not_converged"])
    line = {
        "metric": "Sinkhorn-EM cost-entries/s",
        "value": entries / dt,
        "unit": "cost-entries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: Sinkhorn-EM iterations on {preset.n_grains} "
                               f"{'BCC' if preset.centering == 'I' else 'FCC'} grains (a = {preset.a} A), "
                               f"{preset.n_rot} rotations x {preset.domega_deg} deg, sigma {preset.sigma_mm} mm, "
                               f"{int(100 * preset.outlier_frac)}% outliers",
                   "detected_spots": obs.n, "model_spots": model.n,
                   "entries_per_pass": int(np.sum(blk_i * blk_j)),
                   "em_iterations": [0, args.steps], "schedule_length": n_sched,
                   "schedule": f"{preset.n_stages} stages x {preset.iters_per_stage} EM iterations, "
                               f"{preset.eps_start:.4g} -> {preset.eps_end:.4g} mm^2; one run from the start, "
                               f"iterations beyond it at the last temperature",
                   "sinkhorn_tol": 1e-5, "k_gn": 2},
        "em_iters_per_s": args.steps / dt,
        "sinkhorn_iters": int(sum(s["sinkhorn_iters"] for s in stats)),
        "sinkhorn_capped": int(sum(s["not_converged"] for s in stats)),
        "stages": stages,
        "recall_after_run": recall(qf, xf, q_true, x_true) / len(q_true),
        "tile": {"requested": args.tile, "two_per_lane_solves": int(sum(s["tile2_solves"] for s in stats)),
                 "solves": len(stats)},
        "roofline": {"kernel": "Sinkhorn row/column pass (k_row, k_col)", "bound": "alu",
                     "achieved": achieved / 1e9, "peak": PEAK_ENTRIES_PER_S / 1e9,
                     "unit": "Gentries/s", "frac": achieved / PEAK_ENTRIES_PER_S,
                     "traffic": ROW_PASS_HBM_BYTES if args.workload == "learned" else None,
                     "traffic_unit": "HBM bytes per row-pass launch",
                     "per_entry": {"valu": ALGO_VALU_PER_ENTRY, "trans": ALGO_TRANS_PER_ENTRY,
                                   "counted_as": "the method's algorithmic work per entry"},
                     "compiled": {"valu": VALU_PER_ENTRY, "trans": TRANS_PER_ENTRY,
                                  "peak": PEAK_COMPILED_ENTRIES_PER_S / 1e9,
                                  "frac": achieved / PEAK_COMPILED_ENTRIES_PER_S},
                     "passes": sk_pass, "avg_pass_ms": sk_ms / max(sk_pass, 1)},
        "mstep": {"ms": sum(s["mstep_ms"] for s in stats),
                  "entries": int(sum(s["mstep_entries"] for s in stats))},
    }
    log = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
    if not args.no_forward:
        line["forward_model"] = bench_forward(laue, args.forward_grains, log)
    if not args.no_batching:
        line["batching"] = bench_batching(laue, args.batch_samples, 3, log)
    if not args.no_sparse:
        line["sparse_assignment"] = bench_sparse(laue, preset, args.sparse_rho, args.sparse_iters, log)
    if not args.no_unbalanced:
        kl = [tuple(float(v) for v in item.split(",")) for item in args.unbalanced_kl.split(";")]
        import inputgen as ig
        fracs = [float(v) for v in args.partial_fracs.split(",") if v]
        line["outlier_models"] = bench_outlier_models(laue, ig.PRESETS[args.unbalanced_workload], kl, fracs,
                                                      args.unbalanced_iters, log)
        line["outlier_models"]["workload"] = args.unbalanced_workload
    if not args.no_mstep_methods:
        import inputgen as ig
        line["mstep_methods"] = bench_mstep_methods(laue, preset, ig.PRESETS["medium"], args.steps, log)
    if not args.no_index:
        line["time_to_index"] = {}
        for item in [x for x in args.index_workloads.split(";") if x.strip()]:
            wl, o = parse_index_line(item)
            key = o.get("name", f"{wl}.{o['recipe']}")
            line["time_to_index"][key] = bench_index(
                laue, wl, o["pairs"], o["lpairs"], log, sobol_points=o["sobol"], recipe=o["recipe"],
                max_candidates=o["cand"], plain_max=o["pcand"], train_examples=o["examples"],
                spot_per_candidate=o["spot"], rho=o["rho"])
    if args.index_limits:
        import inputgen as ig
        line["index_limits"] = {wl: bench_index_limits(laue, ig.PRESETS[wl], log)
                                for wl in args.index_limits.split(",") if wl}
    if not args.no_cpu_baseline:
        cb = cpu_baseline(preset)
        runs = cpu_oracle_runs()
        cb["oracle_runs"] = runs
        cb["oracle_extrapolated"] = cpu_extrapolate(line, cb, runs)
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
