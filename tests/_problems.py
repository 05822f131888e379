"""Seeded synthetic problems for the parity tests: everything here is built by
the oracle (simulation, model-spot sets, FP32-rounded column data) and then
handed, unchanged, to both the oracle and the HIP library."""
from __future__ import annotations

import dataclasses

import numpy as np

import inputgen as ig
from oracle import cost, crystal, forward, simulate


@dataclasses.dataclass
class Problem:
    preset: object
    planes: dict
    geom: object
    q_true: np.ndarray
    x_true: np.ndarray
    obs: dict            # p12 (FP32-exact FP64), block, offsets, grain, plane
    q0: np.ndarray
    x0: np.ndarray
    model: dict          # oracle model-spot set at (q0, x0) with offsets
    s12: np.ndarray      # FP32-exact column data at (q0, x0)
    vloc: np.ndarray


def make(preset, n_rot=None, n_grains=None, sigma=None, frac=None, seed_shift=0, perturb=(0.5, 0.5)):
    p = preset
    pl = crystal.cubic_planes(p.a, p.centering, p.n_max)
    geom = forward.Geometry(p.n_rot if n_rot is None else n_rot, np.deg2rad(p.domega_deg),
                            p.detectors, p.lam_min, p.lam_max)
    q, x = ig.random_grains(p, n=n_grains, seed=p.seed + seed_shift)
    sim = simulate.simulate(pl, q, x, geom, p.sigma_mm if sigma is None else sigma,
                            p.outlier_frac if frac is None else frac, p.seed + seed_shift, p.distance)
    sim["p12"] = ig.to_f32_exact(sim["p12"])
    q0, x0 = ig.perturb_grains(q, x, perturb[0], perturb[1], p.seed + 17 + seed_shift)
    model = forward.enumerate_visible(pl, q0, x0, geom)
    model["offsets"] = forward.block_offsets(model["block"], geom.n_blocks)
    ev = forward.eval_fixed(pl, q0, x0, geom, model["m"], model["n"], model["t"], model["det"])
    s12 = ig.to_f32_exact(ev["s12"])
    vloc = ig.to_f32_exact(cost.v_local(geom, model["det"], ev["v"]))
    return Problem(p, pl, geom, q, x, sim, q0, x0, model, s12, vloc)


def oracle_costs(P):
    C = []
    off, mo = P.obs["offsets"], P.model["offsets"]
    for b in range(P.geom.n_blocks):
        C.append(cost.chord_cost(P.obs["p12"][off[b]:off[b + 1]], P.s12[mo[b]:mo[b + 1]],
                                 P.vloc[mo[b]:mo[b + 1]], P.preset.distance))
    return C


def gpu_objects(laue, P):
    """Geometry, planes, detected spots and model spots (with the FP32 column
    data of the problem) for the HIP library."""
    p = P.preset
    geom = laue.make_geometry(P.geom.n_rot, np.deg2rad(p.domega_deg), p.detectors, p.lam_min, p.lam_max)
    planes = laue.laue_planes_cubic(p.a, p.centering, p.n_max)
    obs = laue.ObsSpots.from_numpy(P.obs["p12"], P.obs["offsets"])
    m = P.model
    model = laue.ModelSpots.from_arrays(P.geom.n_blocks, m["offsets"], m["m"], m["n"], m["block"],
                                        P.s12[:, 0], P.s12[:, 1], P.vloc[:, 0], P.vloc[:, 1],
                                        P.vloc[:, 2])
    return geom, planes, obs, model


def tied_rows(P, rho, rel=1e-5, abs_=1e-5):
    """Detected spots whose rho-nearest model-spot set is decided by a near-tie:
    the rho-th and (rho+1)-th smallest FP64 costs of the row lie within the
    FP32 cost accuracy of each other, so an FP32 evaluation may pick either."""
    out = []
    off = P.obs["offsets"]
    for b, Cb in enumerate(oracle_costs(P)):
        k = min(int(rho), Cb.shape[1])
        if k == 0 or k == Cb.shape[1]:
            continue
        s = np.sort(Cb, axis=1)
        gap = s[:, k] - s[:, k - 1]
        out.extend(off[b] + np.flatnonzero(gap <= rel * s[:, k - 1] + abs_))
    return np.array(out, dtype=np.int64)


def without_tied_rows(P, rho):
    """The problem with the near-tied detected spots of tied_rows removed (the
    other rows keep their sets: a row's set depends on its own costs only)."""
    drop = tied_rows(P, rho)
    if drop.size == 0:
        return P
    n = P.obs["p12"].shape[0]
    keep = np.ones(n, bool)
    keep[drop] = False
    obs = {k: (v[keep] if isinstance(v, np.ndarray) and v.shape[:1] == (n,) else v) for k, v in P.obs.items()}
    nb = P.geom.n_blocks
    obs["offsets"] = forward.block_offsets(obs["block"], nb)
    obs["n_true"] = np.bincount(obs["block"][obs["grain"] >= 0], minlength=nb).astype(np.int64)
    return dataclasses.replace(P, obs=obs)
