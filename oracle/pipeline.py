"""End-to-end indexing of the oracle: the multigrain solve (paper Sec. 6,
Alg. MultiGrainLaueOT) with spot-pair candidates as the starts.

Test infrastructure: FP64, plain NumPy; each step is the oracle function of
its stage, taken in the paper's order:
  1. candidates of the first n_pairs spot pairs (oracle/candidates.py), at most
     max_candidates of them, the first ones;
  2. learned mode only: the caller's candidate ranking, the ceil(top_frac n)
     best by oracle/proposal.select_top;
  3. every chosen candidate refined from (q, x = 0) and scored
     (oracle/single.py); a candidate with model spots is kept when its
     unmatched count is below f_out times its model spots; dropped
     candidates get an empty SPOT column;
  4. greedy SPOT with the outlier floor and k* at the largest drop of the
     increment over 8 picks (single.n_prototypes);
  5. the harmonic-merged model spots of the first k* picks, frozen, and the EM
     of oracle/em.py with T_b = max(ceil(t_b_frac |J|), |J| - |I|).
With starts = (q, x) (the Sobol grid of Sec. 6.1, oracle/sobol.py) those
replace steps 1-2: every start is refined from its own (q, x).
"""
from __future__ import annotations

import math

import numpy as np

from . import candidates, em, forward, proposal, single


def index(planes, geom, distance, p12, offsets, sigma, c_out, eps_list, n_pairs, seed, delta_deg=1.5,
          max_candidates=None, k_refine=8, k_gn_refine=1, f_out=0.1, k_max=None, t_b_frac=0.4, k_gn=2,
          ranking=None, top_frac=0.05, starts=None, refine_eps=None, zeta_tol=None, n_final_max=0):
    """refine_eps: the single-grain temperature list (None: single.refine's
    default); zeta_tol, n_final_max: Alg. LaueOT's plan-change stop at the last
    EM temperature (em.run)."""
    if starts is not None:
        cand = {"q": np.asarray(starts[0], dtype=np.float64), "x": np.asarray(starts[1], dtype=np.float64)}
    else:
        cand = candidates.generate(planes, geom, p12, offsets, n_pairs, seed, delta_deg)
    n = len(cand["q"])
    if max_candidates is not None:
        n = min(n, int(max_candidates))
    chosen = np.arange(n)
    if ranking is not None:
        chosen = proposal.select_top(np.asarray(ranking)[:n], top_frac)
    n_obs = int(offsets[-1])
    cols, refined = [], []
    for c in chosen:
        x_start = cand["x"][c] if "x" in cand else np.zeros(3)
        q, x, mod = single.refine(planes, geom, distance, p12, offsets, cand["q"][c], x_start, sigma, c_out,
                                  k_refine=k_refine, k_gn=k_gn_refine, eps_list=refine_eps)
        un, nm, rows, vals = single.score(planes, geom, distance, p12, offsets, mod, q, x, sigma, c_out)
        keep = nm > 0 and un < f_out * nm
        cols.append((rows, vals) if keep else (np.zeros(0, np.int64), np.zeros(0)))
        refined.append((q, x))
    phi = -c_out / (2.0 * sigma ** 2)
    picks, gains = single.greedy(cols, n_obs, phi, k_max)
    k = single.n_prototypes(gains)
    out = {"candidates": cand, "chosen": chosen, "picks": picks, "gains": gains, "k": k}
    if k == 0:
        out.update(q=np.zeros((0, 4)), x=np.zeros((0, 3)))
        return out
    q0 = np.array([refined[p][0] for p in picks[:k]])
    x0 = np.array([refined[p][1] for p in picks[:k]])
    model = forward.enumerate_visible(planes, q0, x0, geom)
    model["offsets"] = forward.block_offsets(model["block"], geom.n_blocks)
    J = len(model["m"])
    t_b = max(math.ceil(t_b_frac * J), J - n_obs)
    res = em.run(planes, geom, distance, p12, offsets, model, q0, x0, eps_list, c_out, t_b=t_b, k_gn=k_gn,
                 zeta_tol=zeta_tol, n_final_max=n_final_max)
    out.update(q=res["q"], x=res["x"], q_proto=q0, x_proto=x0, n_model=J, t_b=t_b, em_stats=res["stats"])
    return out
