"""Multigrain Sinkhorn-EM driver of the oracle (paper Sec. 5, Alg. LaueOT).

Test infrastructure: FP64, plain NumPy.

Each EM iteration: model rays and spots of the frozen model-spot list at the
current grains (Alg. LaueOT, first step; the list itself is fixed at the
prototypes, Sec. 4.2), costs, the E-step Sinkhorn (oracle/sinkhorn.py), then
the M-step (oracle/mstep.py) with the plan held fixed.  The annealing
(Sec. 5.1) runs on a temperature list given by the caller: either a fixed
geometric schedule of n_stages stages, iters_per_stage EM iterations each,
eps_s = eps_0 (eps_end/eps_0)^(s/(S-1)) (eps_schedule), or the paper's
cooling by a constant factor per EM iteration down to a floor
(cooling_schedule), followed by iterations at the last temperature until the
plan stops changing (run's zeta_tol).  Sinkhorn potentials are carried over
between iterations (warm start).
"""
from __future__ import annotations

import numpy as np

from . import cost, forward, mstep, partial, sinkhorn, sparse, unbalanced


def eps_schedule(eps0, eps_end, n_stages, iters_per_stage):
    if n_stages == 1:
        stages = [eps0]
    else:
        stages = [eps0 * (eps_end / eps0) ** (s / (n_stages - 1)) for s in range(n_stages)]
    return [e for e in stages for _ in range(iters_per_stage)]


def cooling_schedule(eps_init, eps_floor, cool=0.97):
    """Temperatures of Alg. LaueOT's deterministic annealing (Sec. 5.1, Sec. 7):
    the temperature is multiplied by cool after every EM iteration while it is
    above the floor.  In the paper's units the floor is 1 (eps_p = 1 recovers
    plain EM); on costs in mm^2 it is 2 sigma_mm^2.  Reading of the loop's end
    (the printed test "eps >= 1" never fails once eps stops at a value >= 1):
    the temperatures eps_init cool^k for k = 0 .. K, K the first k with
    eps_init cool^k <= eps_floor; the EM then keeps the last one and iterates
    until the plan stops changing (run(..., zeta_tol=...))."""
    if not (0.0 < cool < 1.0) or eps_init <= 0.0 or eps_floor <= 0.0:
        raise ValueError("need 0 < cool < 1 and positive temperatures")
    out = [float(eps_init)]
    while out[-1] > eps_floor:
        out.append(out[-1] * cool)
    return out


def obs_lab(geom, p12, block):
    det = np.asarray(block) % geom.n_det
    return geom.det_center[det] + p12[:, :1] * geom.det_a1[det] + p12[:, 1:2] * geom.det_a2[det]


def build_costs(planes, geom, distance, p12, obs_off, model, q, x):
    """Column data at (q, x) and the cost blocks."""
    ev = forward.eval_fixed(planes, q, x, geom, model["m"], model["n"], model["t"], model["det"])
    vloc = cost.v_local(geom, model["det"], ev["v"])
    col_off = model["offsets"]
    C = []
    for b in range(geom.n_blocks):
        i0, i1 = obs_off[b], obs_off[b + 1]
        j0, j1 = col_off[b], col_off[b + 1]
        C.append(cost.chord_cost(p12[i0:i1], ev["s12"][j0:j1], vloc[j0:j1], distance))
    return C, ev, vloc


def grain_pairs(planes, geom, p_lab, obs_off, model, Qb, n_grains):
    """Pairs of every grain: (detected spot, model spot of that grain, Q_ij),
    with the model spot's plane index."""
    per = [([], [], [], [], []) for _ in range(n_grains)]
    col_off = model["offsets"]
    for b in range(geom.n_blocks):
        i0, i1 = obs_off[b], obs_off[b + 1]
        j0, j1 = col_off[b], col_off[b + 1]
        if i1 == i0 or j1 == j0:
            continue
        for jj in range(j1 - j0):
            j = j0 + jj
            n = model["n"][j]
            P, T, W, Q, Mi = per[n]
            P.append(p_lab[i0:i1])
            T.append(np.full(i1 - i0, model["t"][j]))
            W.append(np.repeat(planes["w"][model["m"][j]][None], i1 - i0, axis=0))
            Q.append(Qb[b][:, jj])
            Mi.append(np.full(i1 - i0, model["m"][j]))
    out = []
    for P, T, W, Q, Mi in per:
        if P:
            out.append(mstep.Pairs(np.concatenate(P), np.concatenate(T), np.concatenate(W), np.concatenate(Q),
                                   np.concatenate(Mi)))
        else:
            out.append(None)
    return out


def plan_change(Qb_new, bins_new, Qb_old, bins_old):
    """zeta = ||Q^{k+1} - Q^k||_F over the whole plan (blocks and the outlier
    row, column and corner), Alg. LaueOT's stopping quantity."""
    s = sum(float(np.sum((a - b) ** 2)) for a, b in zip(Qb_new, Qb_old))
    s += sum(float(np.sum((np.asarray(a) - np.asarray(b)) ** 2)) for a, b in zip(bins_new, bins_old))
    return float(np.sqrt(s))


def run(planes, geom, distance, p12, obs_off, model, q0, x0, eps_list, c_out, c_unm=0.0,
        c_sink=None, t_b=None, k_gn=2, tol=1e-5, n_max=2000, record=False, rho=None,
        unbalanced_kl=None, mstep_method="gn", paper_kw=None, partial_frac=None,
        zeta_tol=None, n_final_max=0):
    """Run the EM.  model: dict with m, n, t, det (block-sorted) and offsets.
    rho: keep only each detected spot's rho nearest model spots, re-chosen at
    every EM iteration from that iteration's costs (oracle/sparse.py).
    unbalanced_kl: (kappa, lambda) replaces the E-step by unbalanced OT
    (oracle/unbalanced.py; no bins, so c_out, c_unm, c_sink and t_b are
    unused and f0, g0 come back as -inf).
    partial_frac: m_OT replaces the E-step by partial OT (oracle/partial.py,
    started from the Gibbs kernel at every iteration; no bins).
    mstep_method: "gn" (k_gn joint Gauss-Newton steps) or "paper" (k_gn
    coordinate-descent sweeps of LauePosNewton then LaueRotMM,
    mstep.paper_step with the keyword arguments paper_kw).
    zeta_tol, n_final_max (outlier row and column only): after the listed
    temperatures, keep the last one and run up to n_final_max more EM
    iterations, stopping after the first whose plan differs from the previous
    iteration's by zeta = ||Q^{k+1} - Q^k||_F <= zeta_tol (Alg. LaueOT's
    stopping rule at the final temperature; zeta is also recorded for every
    iteration after the first).

    Returns dict with q, x, f, g, f0, g0 and per-iteration stats."""
    c_sink = c_out if c_sink is None else c_sink
    J = len(model["m"])
    t_b = sinkhorn.default_tb(J) if t_b is None else t_b
    q = np.array(q0, dtype=np.float64).copy()
    x = np.array(x0, dtype=np.float64).copy()
    N = q.shape[0]
    p_lab = obs_lab(geom, p12, np.repeat(np.arange(geom.n_blocks), np.diff(obs_off)))
    f = g = None
    f0 = g0 = 0.0
    stats = []
    prev = None
    eps_all = list(eps_list)
    if zeta_tol is not None and eps_all:
        eps_all = eps_all + [eps_all[-1]] * int(n_final_max)
    for it, eps in enumerate(eps_all):
        C, _, _ = build_costs(planes, geom, distance, p12, obs_off, model, q, x)
        if partial_frac is not None:
            Cm = sparse.masked_blocks(C, rho) if rho else C
            sol = partial.solve(Cm, eps, partial_frac, tol=tol, n_max=n_max)
            f, g, f0, g0 = sol["f"], sol["g"], -np.inf, -np.inf
            Qb = partial.plan_blocks(Cm, f, g, eps)
        elif unbalanced_kl is not None:
            Cm = sparse.masked_blocks(C, rho) if rho else C
            sol = unbalanced.solve(Cm, eps, unbalanced_kl[0], unbalanced_kl[1], tol=tol, n_max=n_max, f=f, g=g)
            f, g, f0, g0 = sol["f"], sol["g"], -np.inf, -np.inf
            Qb = unbalanced.plan_blocks(Cm, f, g, eps)
        else:
            P = sinkhorn.Problem(C, c_out, c_unm, c_sink, t_b)
            if rho:
                P = sparse.masked_problem(P, rho)
            sol = sinkhorn.solve(P, eps, tol=tol, n_max=n_max, f=f, g=g, f0=f0, g0=g0)
            f, g, f0, g0 = sol["f"], sol["g"], sol["f0"], sol["g0"]
            Qb = sinkhorn.plan_blocks(P, f, g, eps)
        pairs = grain_pairs(planes, geom, p_lab, obs_off, model, Qb, N)
        steps = np.zeros((N, 6))
        for k in range(k_gn):
            for n in range(N):
                if pairs[n] is None:
                    continue
                if mstep_method == "paper":
                    qn, xn = mstep.paper_step(pairs[n], q[n], x[n], geom, **(paper_kw or {}))
                    steps[n] = np.concatenate([[np.linalg.norm(qn - q[n])], xn - x[n], [0.0, 0.0]])
                    q[n], x[n] = qn, xn
                else:
                    q[n], x[n], st, _, _, _ = mstep.gn_step(pairs[n], q[n], x[n], geom, distance)
                    steps[n] = st
        rec = {"eps": eps, "n_iter": sol["n_iter"], "err": sol["err"],
               "step_max": float(np.max(np.linalg.norm(steps, axis=1))) if N else 0.0}
        if partial_frac is None and unbalanced_kl is None:
            bins = (np.exp((f + g0 - P.c_out) / eps), np.exp((f0 + g - P.c_unm) / eps),
                    np.array([np.exp((f0 + g0 - P.c_sink) / eps)]))
            if prev is not None:
                rec["zeta"] = plan_change(Qb, bins, prev[0], prev[1])
            prev = (Qb, bins)
        if record:
            rec["q"] = q.copy()
            rec["x"] = x.copy()
        stats.append(rec)
        if zeta_tol is not None and it >= len(eps_list) - 1 and rec.get("zeta", np.inf) <= zeta_tol:
            break
    return {"q": q, "x": x, "f": f, "g": g, "f0": f0, "g0": g0, "stats": stats, "t_b": t_b}
