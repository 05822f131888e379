"""Benchmark: Sinkhorn-EM cost-entries/s on one MI355X.

Workload (default "learned-scale"): 1000 BCC grains (a = 2.87 A, planes with
h^2+k^2+l^2 <= 30, band 1-4 A), 60 rotations of 3 deg, two 200 mm detectors at
150 mm, sigma = 1 mm, 70% outliers; detected spots simulated on the GPU; EM
started from the true grains turned by 0.5 deg and moved by 0.5 mm; the
temperature schedule 111 sigma^2 -> 1.11 sigma^2 mm^2 over 5 stages x 4 EM
iterations; Sinkhorn to a relative row-marginal error of 1e-5 (cap 2000).

A step is one EM iteration through the whole path: forward evaluation of the
frozen model spots, the streamed Sinkhorn E-step to tolerance, and two
Gauss-Newton M-step passes.  W warm-up steps run the first W iterations of
the schedule; the K timed steps continue it (wrapping after 20).  The value is
the number of same-block (detected, model) pairs streamed through
cost -> exp -> accumulate in the timed region divided by its wall time.

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
PEAK_ENTRIES_PER_S = VALU_LANE_OPS_PER_S / (VALU_PER_ENTRY + 4 * TRANS_PER_ENTRY)


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


def cpu_baseline(preset, n_rows=10000, chunk=1000):
    """The FP64 oracle on a bounded sample: the row half of one Sinkhorn
    iteration (chord cost + log-sum-exp) for n_rows detected spots of the
    largest block of one projection, in row chunks."""
    import inputgen as ig
    from oracle import cost, crystal, forward, simulate, sinkhorn
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
    rows = ig.to_f32_exact(sim["p12"][sim["offsets"][b]:sim["offsets"][b + 1]])[:n_rows]
    c_out = cost.c_out(preset.sigma_mm, preset.distance)
    gpot = np.zeros(len(s12))
    t0 = time.perf_counter()
    n_ent = 0
    for r in range(0, len(rows), chunk):
        C = cost.chord_cost(rows[r:r + chunk], s12, vl, preset.distance)
        P = sinkhorn.Problem([C], c_out, 0.0, c_out, float(C.shape[1]))
        sinkhorn.row_half(P, gpot, 0.0, preset.eps_start)
        n_ent += C.size
    dt = time.perf_counter() - t0
    return {"value": n_ent / dt, "unit": "cost-entries/s", "cores": 1, "kind": "oracle",
            "sample": f"row half-pass (chord cost + log-sum-exp, FP64 NumPy, one process) over "
                      f"{len(rows)} detected x {len(s12)} model spots of one backscatter block "
                      f"({n_ent:.3g} entries, {dt:.1f} s)",
            "host": platform.processor() or platform.machine(), "os_cpu_count": os.cpu_count(),
            "numpy": np.__version__}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="learned", choices=["learned", "medium"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
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
    # outlier cost: the likelihood of a 3-sigma angular miss, in mm^2
    c_out = 2.0 * preset.distance ** 2 * (1.0 - math.cos(3.0 * preset.sigma_mm / preset.distance))
    t_b = float(math.ceil(0.4 * model.n))
    n_sched = preset.n_stages * preset.iters_per_stage
    eps_list = [preset.eps_start * (preset.eps_end / preset.eps_start) ** (s / (preset.n_stages - 1))
                for s in range(preset.n_stages) for _ in range(preset.iters_per_stage)]
    dev = torch.device("cuda", 0)
    f = torch.zeros(obs.n, dtype=torch.float32, device=dev)
    g = torch.zeros(model.n, dtype=torch.float32, device=dev)
    pot = {"f0": 0.0, "g0": 0.0}

    def step(k):
        eps = eps_list[k % n_sched]
        ot = laue.ot_params(eps, preset.distance, c_out, t_b, tol=1e-5, n_max=2000)
        par = laue.em_params(ot, eps, eps, 1, 1, k_gn=2)
        out = laue.laue_em(geom, planes, obs, model, par, grains, f, g, pot["f0"], pot["g0"], assign=False)
        pot["f0"], pot["g0"] = out["f0"], out["g0"]
        return out

    print(f"bench: {args.workload}: {obs.n} detected, {model.n} model spots, "
          f"{int(np.sum(np.diff(obs.block_off) * np.diff(model.block_off)))} entries per pass",
          file=sys.stderr, flush=True)
    for k in range(args.warmup):
        o = step(k)
        print(f"bench: warm-up step {k}: {o['sinkhorn_iters']} Sinkhorn iterations", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        stats.append(step(k))
        print(f"bench: step {k}: eps {eps_list[k % n_sched]:.3g}, {stats[-1]['sinkhorn_iters']} Sinkhorn "
              f"iterations, {stats[-1]['sinkhorn_ms']:.1f} ms in Sinkhorn passes", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    entries = sum(s["cost_entries"] for s in stats)
    sk_ms = sum(s["sinkhorn_ms"] for s in stats)
    sk_ent = sum(s["sinkhorn_entries"] for s in stats)
    sk_pass = sum(s["sinkhorn_passes"] for s in stats)
    achieved = sk_ent / (sk_ms * 1e-3)
    blk_i = np.diff(obs.block_off)
    blk_j = np.diff(model.block_off)
    line = {
        "metric": "Sinkhorn-EM cost-entries/s",
        "value": entries / dt,
        "unit": "cost-entries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: Sinkhorn-EM iterations on {preset.n_grains} BCC grains, "
                               f"{preset.n_rot} rotations x {preset.domega_deg} deg, sigma {preset.sigma_mm} mm, "
                               f"{int(100 * preset.outlier_frac)}% outliers",
                   "detected_spots": obs.n, "model_spots": model.n,
                   "entries_per_pass": int(np.sum(blk_i * blk_j)),
                   "em_iterations": [args.warmup, args.warmup + args.steps],
                   "sinkhorn_tol": 1e-5, "k_gn": 2},
        "em_iters_per_s": args.steps / dt,
        "sinkhorn_iters": int(sum(s["sinkhorn_iters"] for s in stats)),
        "sinkhorn_capped": int(sum(s["not_converged"] for s in stats)),
        "roofline": {"kernel": "Sinkhorn row/column pass (k_row, k_col)", "bound": "alu",
                     "achieved": achieved / 1e9, "peak": PEAK_ENTRIES_PER_S / 1e9,
                     "unit": "Gentries/s", "frac": achieved / PEAK_ENTRIES_PER_S, "traffic": None,
                     "per_entry": {"valu": VALU_PER_ENTRY, "trans": TRANS_PER_ENTRY},
                     "passes": sk_pass, "avg_pass_ms": sk_ms / max(sk_pass, 1)},
        "mstep": {"ms": sum(s["mstep_ms"] for s in stats),
                  "entries": int(sum(s["mstep_entries"] for s in stats))},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(preset)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
