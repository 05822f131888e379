"""Python binding of liblaueot (MI355X LaueOT hot path).

Argument marshalling only: every step runs in the HIP library behind the C
ABI of include/laueot.h.  PyTorch provides device memory and the stream.
Functions carry the names of the C entry points they call.  There is no CPU
fallback: if the library is missing the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import _abi
from ._abi import (laue_assignments, laue_em_params, laue_em_stats, laue_geometry, laue_gn_params,
                   laue_grains, laue_model_spots, laue_obs_spots, laue_ot_params, laue_ot_stats,
                   laue_planes, laue_potentials)

__all__ = ["LaueError", "require_native", "make_geometry", "geometry_from_preset", "Planes",
           "Grains", "ModelSpots", "ObsSpots", "ot_params", "laue_planes_cubic",
           "laue_forward_enumerate", "laue_forward_eval", "laue_simulate", "laue_sinkhorn",
           "laue_plan_block", "laue_cost_block", "laue_mstep", "laue_em", "laue_version"]

_LIB = None


class LaueError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblaueot error {code}: {msg}")
        self.code = code


def require_native():
    """Load liblaueot.so (built in-tree) or raise: there is no fallback path."""
    global _LIB
    if _LIB is None:
        import torch  # noqa: F401  (the HIP runtime of torch must be loaded first)
        if not os.path.exists(_abi.LIB_PATH):
            raise ImportError(f"{_abi.LIB_PATH} is missing: run python -m paper_2404_06478_amd.build")
        _LIB = _abi.load()
    return _LIB


def _check(rc):
    if rc < 0:
        raise LaueError(rc, require_native().laue_last_error().decode())
    return rc


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev():
    import torch
    return torch.device("cuda", torch.cuda.current_device())


def _workspace(nbytes):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=_dev())


def laue_version():
    return require_native().laue_version()


# ---------------------------------------------------------------- geometry

def make_geometry(n_rot, domega, detectors, lam_min, lam_max, omega0=0.0):
    """laue_geometry from detector records with center/normal/axis1/axis2/size."""
    g = laue_geometry()
    g.n_rot, g.n_det = int(n_rot), len(detectors)
    g.omega0, g.domega = float(omega0), float(domega)
    g.lambda_min, g.lambda_max = float(lam_min), float(lam_max)
    for k, d in enumerate(detectors):
        for name in ("center", "normal", "axis1", "axis2"):
            getattr(g.det[k], name)[:] = [float(v) for v in getattr(d, name)]
        g.det[k].half_size = float(d.size) / 2.0
    return g


def geometry_from_preset(p, n_rot=None):
    return make_geometry(p.n_rot if n_rot is None else n_rot, math.radians(p.domega_deg),
                         p.detectors, p.lam_min, p.lam_max)


def n_blocks(geom):
    return geom.n_rot * geom.n_det


# ---------------------------------------------------------------- planes / grains

class Planes:
    def __init__(self, hkl, w, d, prev):
        import torch
        self.hkl = np.asarray(hkl)
        self.w = torch.as_tensor(np.asarray(w, np.float32)).reshape(-1, 3).to(_dev())
        self.d = torch.as_tensor(np.asarray(d, np.float32)).to(_dev())
        self.prev = torch.as_tensor(np.asarray(prev, np.int32)).to(_dev())
        self.n = int(self.d.numel())

    @property
    def struct(self):
        return laue_planes(self.n, self.w.data_ptr(), self.d.data_ptr(), self.prev.data_ptr())


def laue_planes_cubic(a, centering, n_max):
    lib = require_native()
    n = C.c_int32()
    _check(lib.laue_planes_cubic(float(a), centering.encode(), int(n_max), C.byref(n), None, None, None, None))
    hkl = np.zeros((n.value, 3), np.int32)
    w = np.zeros((n.value, 3), np.float32)
    d = np.zeros(n.value, np.float32)
    prev = np.zeros(n.value, np.int32)
    _check(lib.laue_planes_cubic(float(a), centering.encode(), int(n_max), C.byref(n),
                                 hkl.ctypes.data, w.ctypes.data, d.ctypes.data, prev.ctypes.data))
    return Planes(hkl, w, d, prev)


class Grains:
    """FP64 quaternions [n,4] and positions [n,3] on the device."""

    def __init__(self, q, x):
        import torch
        self.q = torch.as_tensor(np.asarray(q, np.float64)).reshape(-1, 4).to(_dev()).contiguous()
        self.x = torch.as_tensor(np.asarray(x, np.float64)).reshape(-1, 3).to(_dev()).contiguous()
        self.n = int(self.q.shape[0])

    @property
    def struct(self):
        return laue_grains(self.n, self.q.data_ptr(), self.x.data_ptr())

    def numpy(self):
        return self.q.cpu().numpy(), self.x.cpu().numpy()


# ---------------------------------------------------------------- spots

class ModelSpots:
    """Block-sorted model spots (device SoA) with host block offsets."""

    FIELDS_I = ("plane", "grain", "block")
    FIELDS_F = ("s1", "s2", "vn", "v1", "v2", "lam")

    def __init__(self, n, nb):
        import torch
        dev = _dev()
        self.n = int(n)
        m = max(self.n, 1)
        for f in self.FIELDS_I:
            setattr(self, f, torch.zeros(m, dtype=torch.int32, device=dev))
        for f in self.FIELDS_F:
            setattr(self, f, torch.zeros(m, dtype=torch.float32, device=dev))
        self.flags = torch.zeros(m, dtype=torch.uint8, device=dev)
        self.block_off = np.zeros(nb + 1, np.int64)

    def struct(self):
        s = laue_model_spots()
        s.n = self.n
        for f in self.FIELDS_I + self.FIELDS_F + ("flags",):
            setattr(s, f, getattr(self, f).data_ptr())
        s.block_off = self.block_off.ctypes.data
        return s

    @classmethod
    def from_arrays(cls, nb, block_off, plane, grain, block, s1=None, s2=None, vn=None, v1=None,
                    v2=None):
        import torch
        m = cls(len(plane), nb)
        m.block_off[:] = np.asarray(block_off, np.int64)
        if m.n:
            for f, v in (("plane", plane), ("grain", grain), ("block", block)):
                getattr(m, f)[:m.n] = torch.as_tensor(np.asarray(v, np.int32))
            for f, v in (("s1", s1), ("s2", s2), ("vn", vn), ("v1", v1), ("v2", v2)):
                if v is not None:
                    getattr(m, f)[:m.n] = torch.as_tensor(np.asarray(v, np.float32))
        return m

    def numpy(self):
        out = {f: getattr(self, f)[:self.n].cpu().numpy() for f in self.FIELDS_I + self.FIELDS_F + ("flags",)}
        out["block_off"] = self.block_off.copy()
        return out


class ObsSpots:
    """Block-sorted detected spots (device FP32) with host block offsets."""

    def __init__(self, p1, p2, block_off, grain=None, plane=None):
        self.p1, self.p2 = p1, p2
        self.block_off = np.asarray(block_off, np.int64).copy()
        self.n = int(self.block_off[-1])
        self.grain, self.plane = grain, plane

    @classmethod
    def from_numpy(cls, p12, block_off):
        import torch
        p12 = np.asarray(p12, np.float32).reshape(-1, 2)
        dev = _dev()
        p1 = torch.as_tensor(np.ascontiguousarray(p12[:, 0])).to(dev)
        p2 = torch.as_tensor(np.ascontiguousarray(p12[:, 1])).to(dev)
        if p1.numel() == 0:
            p1 = torch.zeros(1, dtype=torch.float32, device=dev)
            p2 = torch.zeros(1, dtype=torch.float32, device=dev)
        return cls(p1, p2, block_off)

    def struct(self):
        return laue_obs_spots(self.n, self.p1.data_ptr(), self.p2.data_ptr(), self.block_off.ctypes.data)


def laue_forward_enumerate(geom, planes, grains, merge_harmonics=True):
    lib = require_native()
    ws = _workspace(lib.laue_forward_workspace_size(C.byref(geom), planes.n, grains.n))
    nb = n_blocks(geom)
    probe = ModelSpots(0, nb)
    ps = probe.struct()
    ps.n = 0
    nout = C.c_int64()
    ps_planes, ps_grains = planes.struct, grains.struct
    rc = lib.laue_forward_enumerate(C.byref(geom), C.byref(ps_planes), C.byref(ps_grains),
                                    int(bool(merge_harmonics)), C.byref(ps), C.byref(nout),
                                    _ptr(ws), ws.numel(), _stream())
    if rc == _abi.LAUE_ECAPACITY:
        out = ModelSpots(nout.value, nb)
        s = out.struct()
        rc = lib.laue_forward_enumerate_counted(C.byref(geom), C.byref(ps_planes), C.byref(ps_grains),
                                                int(bool(merge_harmonics)), C.byref(s), C.byref(nout),
                                                _ptr(ws), ws.numel(), _stream())
        _check(rc)
        return out
    _check(rc)
    probe.block_off[:] = np.zeros(nb + 1, np.int64)
    return probe


def laue_forward_count(geom, planes, grains, merge_harmonics=True):
    """Number of visible reflections (the count of laue_forward_enumerate,
    no spot written)."""
    lib = require_native()
    ws = _workspace(lib.laue_forward_workspace_size(C.byref(geom), planes.n, grains.n))
    probe = ModelSpots(0, n_blocks(geom))
    ps = probe.struct()
    ps.n = 0
    nout = C.c_int64()
    rc = lib.laue_forward_enumerate(C.byref(geom), C.byref(planes.struct), C.byref(grains.struct),
                                    int(bool(merge_harmonics)), C.byref(ps), C.byref(nout),
                                    _ptr(ws), ws.numel(), _stream())
    if rc != _abi.LAUE_ECAPACITY:
        _check(rc)
    return int(nout.value)


def laue_forward_eval(geom, planes, grains, model):
    lib = require_native()
    ws = _workspace(lib.laue_forward_workspace_size(C.byref(geom), planes.n, grains.n))
    s = model.struct()
    _check(lib.laue_forward_eval(C.byref(geom), C.byref(planes.struct), C.byref(grains.struct),
                                 C.byref(s), _ptr(ws), ws.numel(), _stream()))
    return model


def laue_simulate(geom, planes, truth, sigma_mm, distance, outlier_frac, seed):
    import torch
    lib = require_native()
    n_true = laue_forward_count(geom, planes, truth, True)
    # capacity: true spots + outliers (frac * n_true rounded per block, + 1 per block)
    cap = int(n_true * (1.0 + outlier_frac)) + n_blocks(geom) + 1
    ws = _workspace(lib.laue_simulate_workspace_size(C.byref(geom), planes.n, truth.n, n_true, cap))
    dev = _dev()
    p1 = torch.zeros(cap, dtype=torch.float32, device=dev)
    p2 = torch.zeros(cap, dtype=torch.float32, device=dev)
    gr = torch.zeros(cap, dtype=torch.int32, device=dev)
    pl = torch.zeros(cap, dtype=torch.int32, device=dev)
    boff = np.zeros(n_blocks(geom) + 1, np.int64)
    nout = C.c_int64(cap)
    _check(lib.laue_simulate(C.byref(geom), C.byref(planes.struct), C.byref(truth.struct),
                             float(sigma_mm), float(distance), float(outlier_frac), int(seed),
                             int(n_true), _ptr(p1), _ptr(p2), _ptr(gr), _ptr(pl),
                             C.c_void_p(boff.ctypes.data), C.byref(nout), _ptr(ws), ws.numel(),
                             _stream()))
    n = nout.value
    return ObsSpots(p1, p2, boff, gr[:max(n, 1)], pl[:max(n, 1)])


# ---------------------------------------------------------------- E / M steps

def ot_params(eps, distance, c_out, t_b, c_unm=0.0, c_sink=None, tol=1e-5, n_max=2000, chunk=0, rho=0,
              unbalanced_kl=None, partial_frac=None):
    """rho: 0 dense; 8, 16 or 32 keeps each detected spot's rho nearest model spots.
    unbalanced_kl: (kappa, lam) in mm^2 selects unbalanced OT (no bins);
    partial_frac: m_OT in (0, 1] selects partial OT (no bins)."""
    p = laue_ot_params()
    p.eps, p.distance, p.c_out, p.c_unm = float(eps), float(distance), float(c_out), float(c_unm)
    p.c_sink = float(c_out if c_sink is None else c_sink)
    p.t_b, p.tol, p.n_max, p.chunk = float(t_b), float(tol), int(n_max), int(chunk)
    p.rho = int(rho)
    if unbalanced_kl is not None:
        p.outlier_model = 1
        p.kappa, p.lam = float(unbalanced_kl[0]), float(unbalanced_kl[1])
    if partial_frac is not None:
        p.outlier_model = 2
        p.m_frac = float(partial_frac)
    return p


def ot_defaults(sigma_mm, distance, n_model):
    """laue_ot_params of the outlier row and column of Sec. 7 (laue_ot_defaults)."""
    lib = require_native()
    p = laue_ot_params()
    _check(lib.laue_ot_defaults(float(sigma_mm), float(distance), int(n_model), C.byref(p)))
    return p


def c_out_3sigma(sigma_mm, distance):
    """The outlier cost of a 3-sigma angular miss (laue_ot_defaults' c_out)."""
    return ot_defaults(sigma_mm, distance, 0).c_out


def _ws_size(geom, n_obs, n_model, n_grains, rho):
    """Workspace bytes of the Sinkhorn / M-step / EM calls of one sample."""
    lib = require_native()
    if not rho:
        return lib.laue_sinkhorn_workspace_size(C.byref(geom), int(n_obs), int(n_model), int(n_grains))
    no = np.array([n_obs], np.int64)
    nm = np.array([n_model], np.int64)
    ng = np.array([n_grains], np.int32)
    return lib.laue_sparse_workspace_size(1, C.byref(geom), C.c_void_p(no.ctypes.data), C.c_void_p(nm.ctypes.data),
                                          C.c_void_p(ng.ctypes.data), int(rho))


def laue_sparse_neighbors(geom, obs, model, ot):
    """Neighbour sets of the sparse assignment: (nbr [n_obs, rho] int32, cost
    [n_obs, rho] FP32 mm^2, kept pairs)."""
    import torch
    lib = require_native()
    dev = _dev()
    rho = int(ot.rho)
    ws = _workspace(_ws_size(geom, obs.n, model.n, 0, rho))
    nbr = torch.empty((max(obs.n, 1), rho), dtype=torch.int32, device=dev)
    cost = torch.empty((max(obs.n, 1), rho), dtype=torch.float32, device=dev)
    npairs = C.c_int64()
    o, m = obs.struct(), model.struct()
    _check(lib.laue_sparse_neighbors(C.byref(geom), C.byref(o), C.byref(m), C.byref(ot), _ptr(nbr), _ptr(cost),
                                     C.byref(npairs), _ptr(ws), ws.numel(), _stream()))
    return nbr[:obs.n], cost[:obs.n], npairs.value


def laue_eps_init(geom, obs, model, ot):
    """The sparse assignment's first temperature (mm^2): median farthest-neighbour cost / ln 100."""
    lib = require_native()
    ws = _workspace(_ws_size(geom, obs.n, model.n, 0, int(ot.rho)))
    out = C.c_double()
    o, m = obs.struct(), model.struct()
    _check(lib.laue_eps_init(C.byref(geom), C.byref(o), C.byref(m), C.byref(ot), C.byref(out), _ptr(ws),
                             ws.numel(), _stream()))
    return out.value


def laue_sinkhorn(geom, obs, model, ot, f, g, f0=0.0, g0=0.0):
    """Runs Sinkhorn in place on f, g (device FP32); returns (f0, g0, stats dict, code)."""
    lib = require_native()
    ws = _workspace(_ws_size(geom, obs.n, model.n, 0, ot.rho))
    pot = laue_potentials(f.data_ptr(), g.data_ptr(), float(f0), float(g0))
    st = laue_ot_stats()
    o, m = obs.struct(), model.struct()
    rc = _check(lib.laue_sinkhorn(C.byref(geom), C.byref(o), C.byref(m), C.byref(ot), C.byref(pot),
                                  C.byref(st), _ptr(ws), ws.numel(), _stream()))
    return pot.f0, pot.g0, {"n_iter": st.n_iter, "converged": bool(st.converged), "err": st.err}, rc


def laue_sinkhorn_noalloc(geom, obs, model, ot, f, g, f0=0.0, g0=0.0):
    """laue_sinkhorn on the library's fixed scratch (no workspace, no device
    allocation); returns (f0, g0, stats dict, code)."""
    lib = require_native()
    pot = laue_potentials(f.data_ptr(), g.data_ptr(), float(f0), float(g0))
    st = laue_ot_stats()
    o, m = obs.struct(), model.struct()
    rc = _check(lib.laue_sinkhorn_noalloc(C.byref(geom), C.byref(o), C.byref(m), C.byref(ot), C.byref(pot),
                                          C.byref(st), _stream()))
    return pot.f0, pot.g0, {"n_iter": st.n_iter, "converged": bool(st.converged), "err": st.err}, rc


def laue_objectives(geom, obs, model, ot, f, g, f0, g0, sigma_mm):
    """FP64 plan summaries (dict: mass, cost_inlier, cost_total, entropy, sem_objective)."""
    lib = require_native()
    ws = _workspace(_ws_size(geom, obs.n, model.n, 0, ot.rho))
    pot = laue_potentials(f.data_ptr(), g.data_ptr(), float(f0), float(g0))
    out = _abi.laue_objective()
    o, m = obs.struct(), model.struct()
    _check(lib.laue_objectives(C.byref(geom), C.byref(o), C.byref(m), C.byref(ot), C.byref(pot), float(sigma_mm),
                               C.byref(out), _ptr(ws), ws.numel(), _stream()))
    return {name: getattr(out, name) for name, _ in _abi.laue_objective._fields_}


def laue_plan_block(geom, obs, model, ot, f, g, block):
    import torch
    lib = require_native()
    b = int(block)
    nI = int(obs.block_off[b + 1] - obs.block_off[b])
    nJ = int(model.block_off[b + 1] - model.block_off[b])
    Q = torch.zeros(max(nI * nJ, 1), dtype=torch.float32, device=_dev())
    pot = laue_potentials(f.data_ptr(), g.data_ptr(), 0.0, 0.0)
    o, m = obs.struct(), model.struct()
    _check(lib.laue_plan_block(C.byref(geom), C.byref(o), C.byref(m), C.byref(ot), C.byref(pot),
                               b, _ptr(Q), _stream()))
    return Q[:nI * nJ].reshape(nI, nJ)


def laue_cost_block(geom, obs, model, distance, block):
    import torch
    lib = require_native()
    b = int(block)
    nI = int(obs.block_off[b + 1] - obs.block_off[b])
    nJ = int(model.block_off[b + 1] - model.block_off[b])
    Cm = torch.zeros(max(nI * nJ, 1), dtype=torch.float32, device=_dev())
    o, m = obs.struct(), model.struct()
    _check(lib.laue_cost_block(C.byref(geom), C.byref(o), C.byref(m), float(distance), b, _ptr(Cm),
                               _stream()))
    return Cm[:nI * nJ].reshape(nI, nJ)


def gn_params(k_gn=2, mu_rel=1e-9, mstep="gn", k_newton=3, k_mm=500, tol_x=1e-6, tol_r=1e-12):
    """M-step parameters: mstep "gn" (k_gn joint Gauss-Newton steps) or
    "paper" (k_gn sweeps of LauePosNewton, at most k_newton steps, then
    LaueRotMM, at most k_mm steps)."""
    if mstep not in ("gn", "paper"):
        raise ValueError("mstep must be 'gn' or 'paper'")
    return laue_gn_params(int(k_gn), float(mu_rel), 1 if mstep == "paper" else 0, int(k_newton), int(k_mm),
                          float(tol_x), float(tol_r))


def laue_mstep(geom, planes, obs, model, ot, f, g, grains, k_gn=2, mu_rel=1e-9, **mstep_kw):
    import torch
    lib = require_native()
    ws = _workspace(_ws_size(geom, obs.n, model.n, grains.n, ot.rho))
    gn = gn_params(k_gn, mu_rel, **mstep_kw)
    pot = laue_potentials(f.data_ptr(), g.data_ptr(), 0.0, 0.0)
    steps = torch.zeros(max(grains.n, 1), dtype=torch.float64, device=_dev())
    o, m = obs.struct(), model.struct()
    _check(lib.laue_mstep(C.byref(geom), C.byref(planes.struct), C.byref(o), C.byref(m),
                          C.byref(ot), C.byref(pot), C.byref(gn), C.byref(grains.struct),
                          _ptr(steps), _ptr(ws), ws.numel(), _stream()))
    return steps[:grains.n]


def em_params(ot, eps_start, eps_end, n_stages, iters_per_stage, k_gn=2, mu_rel=1e-9, launch=0, tile=0,
              eps_cool=0.0, final_iters=0, zeta_tol=0.0, sigma_mm=0.0, **mstep_kw):
    """mstep_kw: the M-step options of gn_params (mstep="paper", k_newton, ...).
    eps_cool in (0, 1): Alg. LaueOT's cooling from eps_start down to eps_end,
    then final_iters more iterations with the plan-change stop zeta_tol;
    sigma_mm > 0: the likelihood of the last plan in the results."""
    p = laue_em_params()
    p.ot = ot
    p.gn = gn_params(k_gn, mu_rel, **mstep_kw)
    p.eps_start, p.eps_end = float(eps_start), float(eps_end)
    p.n_stages, p.iters_per_stage = int(n_stages), int(iters_per_stage)
    p.launch = int(launch)
    p.tile = int(tile)
    p.eps_cool, p.final_iters, p.zeta_tol, p.sigma_mm = float(eps_cool), int(final_iters), float(zeta_tol), \
        float(sigma_mm)
    return p


def _assign_tensors(n_obs, n_model, dev):
    import torch
    n, m = max(n_obs, 1), max(n_model, 1)
    return {"j_star": torch.zeros(n, dtype=torch.int32, device=dev),
            "grain": torch.zeros(n, dtype=torch.int32, device=dev),
            "q_star": torch.zeros(n, dtype=torch.float32, device=dev),
            "q_out": torch.zeros(n, dtype=torch.float32, device=dev),
            "q_unm": torch.zeros(m, dtype=torch.float32, device=dev)}


def _assign_struct(t):
    return laue_assignments(*(t[k].data_ptr() for k in ("j_star", "grain", "q_star", "q_out", "q_unm")))


def _em_stats_dict(st):
    out = {name: getattr(st, name) for name, _ in laue_em_stats._fields_ if name != "objective"}
    out["objective"] = {name: getattr(st.objective, name) for name, _ in _abi.laue_objective._fields_}
    return out


def laue_em(geom, planes, obs, model, par, grains, f=None, g=None, f0=0.0, g0=0.0, assign=True):
    """Full EM; grains are updated in place.  Returns a dict of results."""
    import torch
    lib = require_native()
    dev = _dev()
    f = torch.zeros(max(obs.n, 1), dtype=torch.float32, device=dev) if f is None else f
    g = torch.zeros(max(model.n, 1), dtype=torch.float32, device=dev) if g is None else g
    ws = _workspace(_ws_size(geom, obs.n, model.n, grains.n, par.ot.rho))
    pot = laue_potentials(f.data_ptr(), g.data_ptr(), float(f0), float(g0))
    st = laue_em_stats()
    asg = None
    if assign:
        asg_t = _assign_tensors(obs.n, model.n, dev)
        asg = _assign_struct(asg_t)
    o, m = obs.struct(), model.struct()
    rc = _check(lib.laue_em(C.byref(geom), C.byref(planes.struct), C.byref(o), C.byref(m),
                            C.byref(par), C.byref(grains.struct), C.byref(pot),
                            C.byref(asg) if asg is not None else None, C.byref(st), _ptr(ws),
                            ws.numel(), _stream()))
    out = {"f": f, "g": g, "f0": pot.f0, "g0": pot.g0, "code": rc}
    out.update(_em_stats_dict(st))
    if assign:
        out.update({k: v[:(model.n if k == "q_unm" else obs.n)] for k, v in asg_t.items()})
    return out


# ---------------------------------------------------------------- prototype scoring

def laue_candidates_generate(geom, planes, obs, n_pairs, seed, delta_deg=1.5, capacity=None,
                             with_ids=True, with_feat=True, pairs=None):
    """Spot-pair candidates.  Returns a dict of device tensors (q [n,4] FP64, ...).
    pairs: optional (a, b) int32 device tensors of explicit pairs (n_pairs = len)."""
    import torch
    lib = require_native()
    dev = _dev()
    if pairs is not None:
        n_pairs = int(pairs[0].numel())
    ws = _workspace(lib.laue_candidates_workspace_size(C.byref(geom), planes.n, int(n_pairs)))
    par = _abi.laue_cand_params(int(n_pairs), int(seed), float(delta_deg),
                                None if pairs is None else pairs[0].data_ptr(),
                                None if pairs is None else pairs[1].data_ptr())
    nfound = C.c_int64()
    o = obs.struct()
    probe = _abi.laue_candidates()
    q0 = torch.zeros(4, dtype=torch.float64, device=dev)
    probe.n, probe.q = 0, q0.data_ptr()
    _check(lib.laue_candidates_generate(C.byref(geom), C.byref(planes.struct), C.byref(o), C.byref(par),
                                        C.byref(probe), C.byref(nfound), _ptr(ws), ws.numel(), _stream()))
    n = nfound.value if capacity is None else min(int(capacity), nfound.value)
    m = max(n, 1)
    out = {"q": torch.zeros((m, 4), dtype=torch.float64, device=dev)}
    if with_ids:
        for k in ("pair", "ma", "mb", "spot_a", "spot_b"):
            out[k] = torch.zeros(m, dtype=torch.int32, device=dev)
    if with_feat:
        out["feat"] = torch.zeros((m, 16), dtype=torch.float32, device=dev)
    c = _abi.laue_candidates()
    c.n = n
    c.q = out["q"].data_ptr()
    for k in ("pair", "ma", "mb", "spot_a", "spot_b"):
        setattr(c, k, out[k].data_ptr() if k in out else None)
    c.feat = out["feat"].data_ptr() if "feat" in out else None
    if n > 0:
        _check(lib.laue_candidates_generate(C.byref(geom), C.byref(planes.struct), C.byref(o), C.byref(par),
                                            C.byref(c), C.byref(nfound), _ptr(ws), ws.numel(), _stream()))
    res = {k: v[:n] for k, v in out.items()}
    res["n_found"] = nfound.value
    return res


def score_params(sigma_mm, distance, c_out, f_out=0.1, k_refine=8, k_gn=1, mu_rel=1e-9, chunk=4096,
                 max_spots_per_cand=4096, eps_start=None, eps_end=None, eps_cool=0.0, drop_log2=26.0):
    """Single-grain refinement and scoring parameters.  Temperatures are given
    in units of sigma_mm^2 by the defaults (30 -> 1.11, the oracle's reading)
    or explicitly in mm^2; eps_cool > 0 selects Alg. SingleLaueOT's cooling
    eps_start eps_cool^k; drop_log2 (0: FP32-zero terms only) sets which far
    pairs the refinement passes skip (26: terms too small to change an FP32
    row normaliser)."""
    p = _abi.laue_score_params()
    p.sigma_mm, p.distance, p.c_out, p.f_out = float(sigma_mm), float(distance), float(c_out), float(f_out)
    p.eps_start = float(30.0 * sigma_mm ** 2 if eps_start is None else eps_start)
    p.eps_end = float(1.11 * sigma_mm ** 2 if eps_end is None else eps_end)
    p.k_refine, p.k_gn, p.mu_rel = int(k_refine), int(k_gn), float(mu_rel)
    p.chunk, p.max_spots_per_cand = int(chunk), int(max_spots_per_cand)
    p.eps_cool = float(eps_cool)
    p.drop_log2 = float(drop_log2)
    return p


def laue_score_candidates(geom, planes, obs, cand, par, lbar_cap=None):
    """Refines cand (Grains) in place and scores it.  Returns a dict of tensors."""
    import torch
    lib = require_native()
    dev = _dev()
    n = cand.n
    cap = int(lbar_cap if lbar_cap is not None else max(1024, 64 * obs.n))
    ws = _workspace(lib.laue_score_workspace_size(C.byref(geom), obs.n, C.byref(par)))
    out_t = {"n_model": torch.zeros(max(n, 1), dtype=torch.int32, device=dev),
             "n_unmatched": torch.zeros(max(n, 1), dtype=torch.int32, device=dev),
             "keep": torch.zeros(max(n, 1), dtype=torch.uint8, device=dev),
             "lbar_off": torch.zeros(n + 1, dtype=torch.int64, device=dev),
             "lbar_row": torch.zeros(cap, dtype=torch.int32, device=dev),
             "lbar_val": torch.zeros(cap, dtype=torch.float32, device=dev)}
    so = _abi.laue_score_out()
    for k in ("n_model", "n_unmatched", "keep", "lbar_off", "lbar_row", "lbar_val"):
        setattr(so, k, out_t[k].data_ptr())
    so.lbar_cap = cap
    o = obs.struct()
    _check(lib.laue_score_candidates(C.byref(geom), C.byref(planes.struct), C.byref(o), C.byref(cand.struct),
                                     C.byref(par), C.byref(so), _ptr(ws), ws.numel(), _stream()))
    res = {k: (v[:n] if k in ("n_model", "n_unmatched", "keep") else v) for k, v in out_t.items()}
    res["lbar_row"] = out_t["lbar_row"][:so.lbar_n]
    res["lbar_val"] = out_t["lbar_val"][:so.lbar_n]
    res["lbar_n"] = so.lbar_n
    res["pairs_streamed"] = so.pairs_streamed
    res["pairs_evaluated"] = so.pairs_evaluated
    res["pairs_refine"] = so.pairs_refine
    return res


def laue_spot_greedy(lbar_off, lbar_row, lbar_val, n_cand, n_rows, phi, k_max, compact=True):
    """compact: give the library room for a copy of the entries, which the
    selection compacts (the picks and increments are the same either way)."""
    import torch
    lib = require_native()
    dev = _dev()
    extra = 8 * int(lbar_row.numel()) + 1024 if compact else 0
    ws = _workspace(lib.laue_spot_greedy_workspace_size(int(n_cand), int(n_rows)) + extra)
    picks = torch.zeros(max(int(k_max), 1), dtype=torch.int32, device=dev)
    gains = torch.zeros(max(int(k_max), 1), dtype=torch.float64, device=dev)
    npk = C.c_int32()
    _check(lib.laue_spot_greedy(_ptr(lbar_off), _ptr(lbar_row), _ptr(lbar_val), int(n_cand), int(n_rows),
                                float(phi), int(k_max), _ptr(picks), _ptr(gains), C.byref(npk), _ptr(ws),
                                ws.numel(), _stream()))
    return picks[:npk.value], gains[:npk.value]


# ---------------------------------------------------------------- learned proposal

class Mlp:
    """Device storage of the 16-256-256-1 network (FP32 masters, bf16 copies, Adam moments)."""

    N_IN, N_HID = 16, 256

    def __init__(self, seed=0, params=None):
        import torch
        lib = require_native()
        dev = _dev()
        n = lib.laue_mlp_n_params(self.N_IN, self.N_HID)
        nb = lib.laue_mlp_n_bf16(self.N_IN, self.N_HID)
        self.params = torch.zeros(n, dtype=torch.float32, device=dev)
        self.wbf16 = torch.zeros(nb, dtype=torch.int16, device=dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=dev)
        self.s = _abi.laue_mlp(self.N_IN, self.N_HID, self.params.data_ptr(), self.wbf16.data_ptr(),
                               self.m.data_ptr(), self.v.data_ptr(), 0)
        if params is None:
            _check(lib.laue_mlp_init(C.byref(self.s), int(seed), _stream()))
        else:
            self.params.copy_(torch.as_tensor(np.asarray(params, np.float32)))
            _check(lib.laue_mlp_sync_bf16(C.byref(self.s), _stream()))

    @staticmethod
    def pack(p):
        """FP32 parameter vector from a dict W1, b1, W2, b2, w3, b3."""
        return np.concatenate([np.ravel(p[k]) for k in ("W1", "b1", "W2", "b2", "w3", "b3")]).astype(np.float32)

    @staticmethod
    def unpack(v, n_in=16, n_hid=256):
        v = np.asarray(v, dtype=np.float64)
        o = 0
        out = {}
        for k, shape in (("W1", (n_hid, n_in)), ("b1", (n_hid,)), ("W2", (n_hid, n_hid)),
                         ("b2", (n_hid,)), ("w3", (n_hid,)), ("b3", (1,))):
            size = int(np.prod(shape))
            out[k] = v[o:o + size].reshape(shape)
            o += size
        return out


def laue_mlp_forward(mlp, feat):
    import torch
    lib = require_native()
    n = int(feat.shape[0])
    prob = torch.zeros(max(n, 1), dtype=torch.float32, device=_dev())
    ws = _workspace(lib.laue_mlp_forward_workspace_size(n))
    _check(lib.laue_mlp_forward(C.byref(mlp.s), _ptr(feat.contiguous()), n, _ptr(prob), _ptr(ws), ws.numel(),
                                _stream()))
    return prob[:n]


def laue_mlp_backward(mlp, feat, label):
    import torch
    lib = require_native()
    B = int(feat.shape[0])
    grad = torch.zeros_like(mlp.params)
    ws = _workspace(lib.laue_mlp_train_workspace_size(B))
    loss = C.c_double()
    _check(lib.laue_mlp_backward(C.byref(mlp.s), _ptr(feat.contiguous()), _ptr(label.contiguous()), B,
                                 _ptr(grad), C.byref(loss), _ptr(ws), ws.numel(), _stream()))
    return grad, loss.value


def adam_params(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    return _abi.laue_adam_params(float(lr), float(beta1), float(beta2), float(eps))


def laue_mlp_adam(mlp, grad, ap):
    _check(require_native().laue_mlp_adam(C.byref(mlp.s), _ptr(grad), C.byref(ap), _stream()))


def laue_mlp_train_epoch(mlp, feat, label, batch, seed, epoch, ap):
    """One epoch of Adam on the examples (feat [n, 16], label [n], device FP32)
    in the library's seeded order; returns the mean loss."""
    lib = require_native()
    n = int(feat.shape[0])
    ws = _workspace(lib.laue_mlp_epoch_workspace_size(n, int(batch)))
    loss = C.c_double()
    _check(lib.laue_mlp_train_epoch(C.byref(mlp.s), _ptr(feat), _ptr(label), n, int(batch), int(seed), int(epoch),
                                    C.byref(ap), C.byref(loss), _ptr(ws), ws.numel(), _stream()))
    return loss.value


class MlpTrainer:
    """Holds the training workspace for a fixed batch size."""

    def __init__(self, mlp, batch, ap=None):
        lib = require_native()
        self.mlp, self.batch = mlp, int(batch)
        self.ap = adam_params() if ap is None else ap
        self.ws = _workspace(lib.laue_mlp_train_workspace_size(self.batch))

    def laue_mlp_train_step(self, feat, label):
        loss = C.c_double()
        _check(require_native().laue_mlp_train_step(C.byref(self.mlp.s), _ptr(feat), _ptr(label), self.batch,
                                                     C.byref(self.ap), C.byref(loss), _ptr(self.ws),
                                                     self.ws.numel(), _stream()))
        return loss.value


def _cand_struct(cand):
    c = _abi.laue_candidates()
    c.n = int(cand["q"].shape[0])
    c.q = cand["q"].data_ptr()
    for k in ("pair", "ma", "mb", "spot_a", "spot_b"):
        setattr(c, k, cand[k].data_ptr() if k in cand else None)
    c.feat = cand["feat"].data_ptr() if "feat" in cand else None
    return c


def support_params(radius_mm, n_support_planes):
    return _abi.laue_support_params(float(radius_mm), int(n_support_planes))


def laue_candidate_support(geom, planes, obs, cand, radius_mm, n_support_planes):
    """Fills cand['feat'][:, 14:16] (device) with the cheap-support fractions."""
    lib = require_native()
    par = support_params(radius_mm, n_support_planes)
    ws = _workspace(lib.laue_candidate_support_workspace_size(C.byref(geom), planes.n, obs.n, C.byref(par)))
    o, c = obs.struct(), _cand_struct(cand)
    _check(lib.laue_candidate_support(C.byref(geom), C.byref(planes.struct), C.byref(o), C.byref(c), C.byref(par),
                                      _ptr(ws), ws.numel(), _stream()))


def laue_candidate_labels(cand, spot_grain, truth, max_deg=2.0):
    """(label, misorientation deg) device FP32 tensors of the candidates."""
    import torch
    n = int(cand["q"].shape[0])
    lab = torch.zeros(max(n, 1), dtype=torch.float32, device=_dev())
    mis = torch.zeros(max(n, 1), dtype=torch.float32, device=_dev())
    c = _cand_struct(cand)
    _check(require_native().laue_candidate_labels(C.byref(c), _ptr(spot_grain), int(spot_grain.numel()),
                                                  C.byref(truth.struct), float(max_deg), _ptr(lab), _ptr(mis),
                                                  _stream()))
    return lab[:n], mis[:n]


def laue_candidate_labels_nearest(cand, truth, max_deg=1.0):
    """(label, misorientation in degrees, nearest true grain) per candidate."""
    import torch
    n = int(cand["q"].shape[0])
    dev = _dev()
    lab = torch.zeros(max(n, 1), dtype=torch.float32, device=dev)
    mis = torch.zeros(max(n, 1), dtype=torch.float32, device=dev)
    near = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
    _check(require_native().laue_candidate_labels_nearest(C.byref(_cand_struct(cand)), C.byref(truth.struct),
                                                          float(max_deg), _ptr(lab), _ptr(mis), _ptr(near),
                                                          _stream()))
    return lab[:n], mis[:n], near[:n]


def laue_select_top(score, k):
    """Ascending indices (int32 device) of the k largest scores, ties by index."""
    import torch
    lib = require_native()
    n = int(score.numel())
    out = torch.zeros(max(int(k), 1), dtype=torch.int32, device=_dev())
    ws = _workspace(lib.laue_select_top_workspace_size(n))
    _check(lib.laue_select_top(_ptr(score.contiguous()), n, int(k), _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out[:int(k)]


def laue_pairs_same_grain(geom, obs, spot_grain, n_pairs, seed):
    """(a, b) int32 device tensors of same-grain pairs (-1 where none)."""
    import torch
    lib = require_native()
    a = torch.zeros(max(int(n_pairs), 1), dtype=torch.int32, device=_dev())
    b = torch.zeros_like(a)
    ws = _workspace(lib.laue_pairs_same_grain_workspace_size(C.byref(geom)))
    o = obs.struct()
    _check(lib.laue_pairs_same_grain(C.byref(geom), C.byref(o), _ptr(spot_grain), int(n_pairs), int(seed),
                                     _ptr(a), _ptr(b), _ptr(ws), ws.numel(), _stream()))
    return a[:int(n_pairs)], b[:int(n_pairs)]


# ---------------------------------------------------------------- end-to-end indexing

def sobol_params(x_half, first=0, mrp_half=0.0, restrict_fz=True):
    """laue_sobol_params: x_half (3 half extents of the sample box, mm)."""
    p = _abi.laue_sobol_params()
    p.first, p.mrp_half, p.restrict_fz = int(first), float(mrp_half), 1 if restrict_fz else 0
    for k in range(3):
        p.x_half[k] = float(x_half[k])
    return p


def laue_sobol_starts(par, n_points):
    """Sobol-grid starts: (q [n_kept,4], x [n_kept,3]) device FP64 tensors."""
    import torch
    lib = require_native()
    dev = _dev()
    n = int(n_points)
    q = torch.zeros((max(n, 1), 4), dtype=torch.float64, device=dev)
    x = torch.zeros((max(n, 1), 3), dtype=torch.float64, device=dev)
    ws = _workspace(lib.laue_sobol_workspace_size(n))
    kept = C.c_int64(0)
    _check(lib.laue_sobol_starts(C.byref(par), n, _ptr(q), _ptr(x), C.byref(kept), _ptr(ws), ws.numel(), _stream()))
    return q[:kept.value], x[:kept.value]


def index_params(preset_like, mode="plain", n_pairs=None, seed=0, delta_deg=1.5, max_candidates=None, mlp=None,
                 support_radius=None, n_support_planes=None, top_frac=0.05, score=None, lbar_cap=None, k_max=None,
                 max_model_spots=None, t_b_frac=0.4, em=None, n_obs=0, n_planes=0, sobol=None):
    """laue_index_params from a workload description (sigma_mm, distance, grains,
    rotations, schedule) with capacities sized for it.  mode "plain",
    "learned" or "sobol" (max_candidates Sobol points from sobol, default:
    the whole sample box of the workload)."""
    p = _abi.laue_index_params()
    pl = preset_like
    p.mode = {"plain": _abi.LAUE_INDEX_PLAIN, "learned": _abi.LAUE_INDEX_LEARNED,
              "sobol": _abi.LAUE_INDEX_SOBOL}[mode]
    if mode == "sobol":
        p.sobol = sobol if sobol is not None else sobol_params(
            (pl.radius_mm, pl.radius_mm, 0.5 * pl.height_mm))
    n_pairs = int(n_pairs if n_pairs is not None else 8192)
    p.cand = _abi.laue_cand_params(n_pairs, int(seed), float(delta_deg), None, None)
    p.max_candidates = int(max_candidates if max_candidates is not None else 64 * n_pairs)
    if mlp is not None:
        p.mlp = C.pointer(mlp.s)
        p._mlp_ref = mlp
    radius = 4.0 * pl.sigma_mm if support_radius is None else support_radius
    p.support = support_params(radius, n_planes if n_support_planes is None else n_support_planes)
    p.top_frac = float(top_frac)
    c_out = c_out_3sigma(pl.sigma_mm, pl.distance)
    p.score = score if score is not None else score_params(pl.sigma_mm, pl.distance, c_out)
    p.lbar_cap = int(lbar_cap if lbar_cap is not None else max(1 << 16, 2048 * n_obs))
    p.k_max = int(k_max if k_max is not None else max(8, 2 * pl.n_grains))
    p.max_model_spots = int(max_model_spots if max_model_spots is not None
                            else 64 * pl.n_rot * p.k_max)
    p.t_b_frac = float(t_b_frac)
    if em is None:
        ot = ot_params(1.0, pl.distance, c_out, 0.0)
        em = em_params(ot, pl.eps_start, pl.eps_end, pl.n_stages, pl.iters_per_stage)
    p.em = em
    return p


def laue_index(geom, planes, obs, par, assign=True):
    """End-to-end indexing.  Returns (Grains of the k* prototypes after EM, stats dict, assignments)."""
    import torch
    lib = require_native()
    dev = _dev()
    if par.support.n_support_planes <= 0:
        par.support.n_support_planes = planes.n
    need = lib.laue_index_workspace_size(C.byref(geom), planes.n, obs.n, C.byref(par))
    if need == 0:
        raise LaueError(_abi.LAUE_EINVAL, "invalid index parameters")
    ws = _workspace(need)
    out, q, x, asg_t = _index_outputs(par, obs.n, assign, dev)
    st = _abi.laue_index_stats()
    o = obs.struct()
    rc = _check(lib.laue_index(C.byref(geom), C.byref(planes.struct), C.byref(o), C.byref(par), C.byref(out),
                               C.byref(st), _ptr(ws), ws.numel(), _stream()))
    return _index_result(out, st, q, x, asg_t, obs.n, rc)


def _index_result(out, st, q, x, asg_t, n_obs, rc):
    k = out.n_grains
    stats = {name: getattr(st, name) for name, _ in _abi.laue_index_stats._fields_ if name != "em"}
    stats["em"] = _em_stats_dict(st.em)
    stats["code"] = rc
    g = Grains.__new__(Grains)
    g.q, g.x, g.n = q[:max(k, 1)], x[:max(k, 1)], k
    asg = None if asg_t is None else {kk: v[:n_obs] for kk, v in asg_t.items()}
    return g, stats, asg


def _index_outputs(par, n_obs, assign, dev):
    import torch
    K = int(par.k_max)
    q = torch.zeros((K, 4), dtype=torch.float64, device=dev)
    x = torch.zeros((K, 3), dtype=torch.float64, device=dev)
    out = _abi.laue_index_out()
    out.capacity, out.q, out.x = K, q.data_ptr(), x.data_ptr()
    asg_t = None
    if assign:
        asg_t = _assign_tensors(n_obs, 0, dev)
        del asg_t["q_unm"]
        out.assign = laue_assignments(*(asg_t[k].data_ptr() for k in ("j_star", "grain", "q_star", "q_out")))
    return out, q, x, asg_t


def laue_index_batched(geoms, planes, obs, pars, assign=True):
    """laue_index of independent samples in one call (lists of equal length).
    Returns (code, list of (Grains, stats dict, assignments) per sample)."""
    lib = require_native()
    dev = _dev()
    n = len(geoms)
    for par, pl in zip(pars, planes):
        if par.support.n_support_planes <= 0:
            par.support.n_support_planes = pl.n
    G = (laue_geometry * n)(*geoms)
    PL = (_abi.laue_planes * n)(*[p.struct for p in planes])
    O = (laue_obs_spots * n)(*[o.struct() for o in obs])
    PA = (_abi.laue_index_params * n)(*pars)
    npl = (C.c_int32 * n)(*[p.n for p in planes])
    nob = (C.c_int64 * n)(*[o.n for o in obs])
    need = lib.laue_index_batched_workspace_size(n, G, npl, nob, PA)
    if need == 0:
        raise LaueError(_abi.LAUE_EINVAL, "invalid index parameters")
    ws = _workspace(need)
    outs = [_index_outputs(par, o.n, assign, dev) for par, o in zip(pars, obs)]
    OUT = (_abi.laue_index_out * n)(*[o[0] for o in outs])
    ST = (_abi.laue_index_stats * n)()
    rc = _check(lib.laue_index_batched(n, G, PL, O, PA, OUT, ST, _ptr(ws), ws.numel(), _stream()))
    return rc, [_index_result(OUT[k], ST[k], outs[k][1], outs[k][2], outs[k][3], obs[k].n, rc) for k in range(n)]


def laue_em_batched(geoms, planes, obs, models, pars, grains, assign=True):
    """Batched EM of independent samples (lists of equal length); grains are
    updated in place.  Returns (code, list of per-sample result dicts)."""
    import torch
    lib = require_native()
    dev = _dev()
    n = len(geoms)
    G = (laue_geometry * n)(*geoms)
    PL = (_abi.laue_planes * n)(*[p.struct for p in planes])
    O = (laue_obs_spots * n)(*[o.struct() for o in obs])
    M = (laue_model_spots * n)(*[m.struct() for m in models])
    PA = (laue_em_params * n)(*pars)
    GR = (laue_grains * n)(*[g.struct for g in grains])
    f = [torch.zeros(max(o.n, 1), dtype=torch.float32, device=dev) for o in obs]
    g = [torch.zeros(max(m.n, 1), dtype=torch.float32, device=dev) for m in models]
    POT = (laue_potentials * n)(*[laue_potentials(f[k].data_ptr(), g[k].data_ptr(), 0.0, 0.0) for k in range(n)])
    asg_t = []
    AS = None
    if assign:
        asg_t = [_assign_tensors(o.n, m.n, dev) for o, m in zip(obs, models)]
        AS = (laue_assignments * n)(*[_assign_struct(a) for a in asg_t])
    no = np.array([o.n for o in obs], np.int64)
    nm = np.array([m.n for m in models], np.int64)
    ng = np.array([gg.n for gg in grains], np.int32)
    rho = int(pars[0].ot.rho)
    if rho:
        need = lib.laue_sparse_workspace_size(n, G, C.c_void_p(no.ctypes.data), C.c_void_p(nm.ctypes.data),
                                              C.c_void_p(ng.ctypes.data), rho)
    else:
        need = lib.laue_em_batched_workspace_size(n, G, C.c_void_p(no.ctypes.data), C.c_void_p(nm.ctypes.data),
                                                  C.c_void_p(ng.ctypes.data))
    ws = _workspace(need)
    ST = (laue_em_stats * n)()
    rc = _check(lib.laue_em_batched(n, G, PL, O, M, PA, GR, POT, AS, ST, _ptr(ws), ws.numel(), _stream()))
    out = []
    for k in range(n):
        st = ST[k]
        r = {"f": f[k][:obs[k].n], "g": g[k][:models[k].n], "f0": POT[k].f0, "g0": POT[k].g0}
        r.update(_em_stats_dict(st))
        if assign:
            r.update({kk: v[:(models[k].n if kk == "q_unm" else obs[k].n)] for kk, v in asg_t[k].items()})
        out.append(r)
    return rc, out
