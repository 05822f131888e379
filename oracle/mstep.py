"""Per-grain M-step of the oracle (paper Sec. 4.4, Eq. mstep_obj; App. A-B).

Test infrastructure: FP64, plain NumPy.

For a fixed plan Q the M-step maximises <L, Q> over every grain's (R_n, x_n)
separately.  With the cost of oracle/cost.py this is the weighted least
squares problem
    min_{R,x}  sum_ij Q_ij ||rho_ij||^2,   rho_ij = D (rhat_ij(x) - r_j(R)),
since ||rho||^2 = c_ij.  Gauss-Newton over theta = (omega, dx), with the
left perturbation R <- exp([omega]_x) R and x <- x + dx.  The Jacobians are
derived from Eqs. ray_mnt and s_mnt (u = Gamma_t R w, v = R w, tau = |p - y|,
P = I - rhat rhat^T):
    d rho / d x     = -(D / tau) P Gamma_t
    d rho / d omega = -2 D (u e^T + (u.e) I) Gamma_t [v]_x
Normal equations H = sum Q J^T J + mu I, g = sum Q J^T rho, step -H^-1 g, with
a small Levenberg term mu = 1e-9 tr(H)/6 standing in for the paper's iota.

The paper's own M-step (LauePosNewton: Newton on x with Eqs. xgrad / xhess;
LaueRotMM: majorisation-minimisation on R with Eqs. M0, Mm and Wahba's problem,
Alg. wahba) is implemented too, as an independent route to the same
stationary point.
"""
from __future__ import annotations

import math

import numpy as np

from . import crystal

E = np.array([1.0, 0.0, 0.0])


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def apply_step(q, x, omega, dx):
    """R <- exp([omega]_x) R as a quaternion product; x <- x + dx."""
    th = float(np.linalg.norm(omega))
    if th > 0:
        dq = np.concatenate([[math.cos(th / 2)], math.sin(th / 2) * np.asarray(omega) / th])
    else:
        dq = np.array([1.0, 0.0, 0.0, 0.0])
    qn = qmul(dq, q)
    qn /= np.linalg.norm(qn)
    if qn[0] < 0:
        qn = -qn
    return qn, np.asarray(x, dtype=np.float64) + dx


class Pairs:
    """All (detected spot, model spot) pairs of one grain with their weights.

    p_lab [K,3] detected spot in the lab, t [K] rotation index, w [K,3] plane
    normal (crystal frame), weight [K], m [K] plane index (optional: without
    it, pairs with the same normal count as one plane)."""

    def __init__(self, p_lab, t, w, weight, m=None):
        self.p = np.asarray(p_lab, dtype=np.float64)
        self.t = np.asarray(t)
        self.w = np.asarray(w, dtype=np.float64)
        self.q = np.asarray(weight, dtype=np.float64)
        self.m = None if m is None else np.asarray(m)


def residuals_jacobians(pairs, R, x, geom, distance):
    """rho [K,3] and J [K,3,6] (columns: omega, then x) of every pair."""
    G = geom.G[pairs.t]                                    # [K,3,3]
    v = pairs.w @ R.T                                      # R w
    u = np.einsum("kab,kb->ka", G, v)
    r = E - 2.0 * u[:, :1] * u
    y = np.einsum("kab,b->ka", G, x)
    dvec = pairs.p - y
    tau = np.linalg.norm(dvec, axis=1)
    rh = dvec / tau[:, None]
    rho = distance * (rh - r)
    P = np.eye(3)[None] - rh[:, :, None] * rh[:, None, :]
    Jx = -(distance / tau)[:, None, None] * np.einsum("kab,kbc->kac", P, G)
    A = u[:, :, None] * E[None, None, :] + u[:, :1, None] * np.eye(3)[None]
    Vx = np.array([skew(vv) for vv in v])
    Jw = -2.0 * distance * np.einsum("kab,kbc,kcd->kad", A, G, Vx)
    return rho, np.concatenate([Jw, Jx], axis=2)


def objective(pairs, R, x, geom, distance):
    rho, _ = residuals_jacobians(pairs, R, x, geom, distance)
    return float(np.sum(pairs.q * np.einsum("ka,ka->k", rho, rho)))


def normal_equations(pairs, R, x, geom, distance):
    rho, J = residuals_jacobians(pairs, R, x, geom, distance)
    H = np.einsum("k,kai,kaj->ij", pairs.q, J, J)
    g = np.einsum("k,kai,ka->i", pairs.q, J, rho)
    return H, g


def gn_step(pairs, q, x, geom, distance, mu_rel=1e-9):
    """One Gauss-Newton step.  Returns (q, x, step [6], H, g, frozen)."""
    R = crystal.quat_to_R(q)
    H, g = normal_equations(pairs, R, x, geom, distance)
    tr = np.trace(H)
    if not np.isfinite(tr) or tr <= 1e-300:
        return np.asarray(q, dtype=np.float64), np.asarray(x, dtype=np.float64), np.zeros(6), H, g, True
    Hd = H + (mu_rel * tr / 6.0) * np.eye(6)
    step = -np.linalg.solve(Hd, g)
    qn, xn = apply_step(q, x, step[:3], step[3:])
    return qn, xn, step, H, g, False


# ---- the paper's coordinate-descent M-step (App. B) ---------------------------

def wahba(a, b, w):
    """Alg. wahba: R minimising sum_k w_k ||a_k - R b_k||^2 over SO(3)."""
    B = np.einsum("k,ka,kb->ab", w, a, b)
    U, _, Vt = np.linalg.svd(B)
    M = np.diag([1.0, 1.0, np.linalg.det(U) * np.linalg.det(Vt)])
    return U @ M @ Vt


def pos_grad_hess(pairs, R, x, geom):
    """Gradient and Hessian in x of F(x) = sum Q rhat^T r (Eqs. xgrad, xhess,
    without the 1/sigma^2 factor, with the chain rule through y = Gamma_t x):
    per pair dF/dy = -(r - a rhat) / tau and
    d2F/dy2 = -(r rhat^T + rhat r^T - 3 a rhat rhat^T + a I) / tau^2, a = rhat.r."""
    G = geom.G[pairs.t]
    v = pairs.w @ R.T
    u = np.einsum("kab,kb->ka", G, v)
    r = E - 2.0 * u[:, :1] * u
    y = np.einsum("kab,b->ka", G, x)
    dvec = pairs.p - y
    tau = np.linalg.norm(dvec, axis=1)
    rh = dvec / tau[:, None]
    a = np.einsum("ka,ka->k", rh, r)
    gy = -(r - a[:, None] * rh) / tau[:, None]
    Hy = -(r[:, :, None] * rh[:, None, :] + rh[:, :, None] * r[:, None, :]
           - 3.0 * a[:, None, None] * rh[:, :, None] * rh[:, None, :]
           + a[:, None, None] * np.eye(3)[None]) / (tau ** 2)[:, None, None]
    gx = np.einsum("k,kba,kb->a", pairs.q, G, gy)
    Hx = np.einsum("k,kba,kbc,kcd->ad", pairs.q, G, Hy, G)
    return gx, Hx


def pos_newton(pairs, R, x, geom, n_iter=50, tol=1e-12):
    """LauePosNewton: x <- x - H^-1 g with g, H of pos_grad_hess, until
    ||dx|| < tol or n_iter steps (the step that meets tol is applied)."""
    x = np.asarray(x, dtype=np.float64).copy()
    for _ in range(n_iter):
        gx, Hx = pos_grad_hess(pairs, R, x, geom)
        dx = np.linalg.solve(Hx, gx)
        x = x - dx
        if np.linalg.norm(dx) < tol:
            break
    return x


def m0_matrices(pairs, x, geom):
    """Eq. M0 per plane m of the grain:
    M0_m = -sum_{pairs of plane m} Gamma_t^T Q (rhat e^T + e rhat^T) Gamma_t.
    Planes are the pairs' plane indices (pairs without them: their normals).
    Returns (plane keys, normals W [P,3], M0 [P,3,3])."""
    G = geom.G[pairs.t]
    y = np.einsum("kab,b->ka", G, x)
    dvec = pairs.p - y
    rh = dvec / np.linalg.norm(dvec, axis=1, keepdims=True)
    keys = (list(pairs.m.tolist()) if pairs.m is not None
            else [tuple(np.round(w, 12)) for w in pairs.w])
    groups = {}
    for k, key in enumerate(keys):
        groups.setdefault(key, []).append(k)
    W, M0s = [], []
    for key, idx in groups.items():
        M0 = np.zeros((3, 3))
        for k in idx:
            qr = pairs.q[k] * rh[k]
            M0 -= G[k].T @ (np.outer(qr, E) + np.outer(E, qr)) @ G[k]
        W.append(pairs.w[idx[0]])
        M0s.append(M0)
    return list(groups), np.array(W), np.array(M0s)


def mm_shift(M0):
    """Eq. Mm: M0 + |iota| I with iota its smallest eigenvalue when negative."""
    lam_min = np.linalg.eigvalsh(M0)[0]
    return M0 + (abs(lam_min) if lam_min < 0 else 0.0) * np.eye(3)


def rot_mm(pairs, R, x, geom, n_iter=2000, tol=1e-13):
    """LaueRotMM: R <- Wahba(M_m R w_m, w_m, 1) (Eq. majmin_step) until
    ||R' - R||_F < tol or n_iter steps."""
    _, W, M0s = m0_matrices(pairs, x, geom)
    Ms = np.array([mm_shift(M0) for M0 in M0s])
    for _ in range(n_iter):
        a = np.einsum("kab,kb->ka", Ms, W @ R.T)
        Rn = wahba(a, W, np.ones(len(W)))
        done = np.linalg.norm(Rn - R) < tol
        R = Rn
        if done:
            break
    return R


def paper_step(pairs, q, x, geom, n_newton=50, tol_x=1e-12, n_mm=2000, tol_r=1e-13):
    """One coordinate-descent sweep of the paper's M-step (Alg. LaueOT):
    LauePosNewton on x with R fixed, then LaueRotMM on R at the new x."""
    R = crystal.quat_to_R(q)
    xn = pos_newton(pairs, R, x, geom, n_iter=n_newton, tol=tol_x)
    Rn = rot_mm(pairs, R, xn, geom, n_iter=n_mm, tol=tol_r)
    qn = crystal.R_to_quat(Rn)
    if qn[0] < 0:
        qn = -qn
    return qn, xn


def mm_objective(pairs, R, x, geom):
    """sum_m w^T R^T M^0_m R w = G(R) - const, the quantity LaueRotMM increases."""
    G = geom.G[pairs.t]
    y = np.einsum("kab,b->ka", G, x)
    dvec = pairs.p - y
    rh = dvec / np.linalg.norm(dvec, axis=1, keepdims=True)
    u = np.einsum("kab,kb->ka", G, pairs.w @ R.T)
    r = E - 2.0 * u[:, :1] * u
    return float(np.sum(pairs.q * np.einsum("ka,ka->k", rh, r)))
