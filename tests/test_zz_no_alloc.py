"""The allocation-free Sinkhorn (laue_sinkhorn_noalloc) against laue_sinkhorn
with a caller workspace: the same potentials, bin potentials, iteration count
and error, bit for bit, on two calls in a row (the second on a smaller
problem, so stale scratch from the first would show), dense and sparse; a
problem beyond the fixed scratch is refused before anything is enqueued."""
import numpy as np
import pytest
import torch

import inputgen as ig
from oracle import cost, sinkhorn
from tests import _problems

pytestmark = pytest.mark.gpu


def _both(laue, P, eps_scale, rho):
    p = P.preset
    geom, planes, obs, model = _problems.gpu_objects(laue, P)
    eps = eps_scale * p.sigma_mm ** 2
    ot = laue.ot_params(eps, p.distance, cost.c_out(p.sigma_mm, p.distance), sinkhorn.default_tb(model.n),
                        tol=1e-5, n_max=2000, rho=rho)
    res = []
    for fn in (laue.laue_sinkhorn, laue.laue_sinkhorn_noalloc):
        f = torch.zeros(max(obs.n, 1), dtype=torch.float32, device="cuda")
        g = torch.zeros(max(model.n, 1), dtype=torch.float32, device="cuda")
        f0, g0, st, rc = fn(geom, obs, model, ot, f, g)
        res.append((f, g, f0, g0, st, rc))
    return res


@pytest.mark.parametrize("rho", [0, 8])
def test_noalloc_equals_workspace_call_twice(gpu_lib, rho):
    laue = gpu_lib
    big = _problems.make(ig.MEDIUM, n_rot=4, n_grains=60, seed_shift=1)
    small = _problems.make(ig.TINY, seed_shift=2)
    assert len(small.obs["p12"]) < len(big.obs["p12"]) and len(small.model["m"]) < len(big.model["m"])
    for P, scale in ((big, 111.0), (small, 11.1)):
        (fa, ga, f0a, g0a, sa, rca), (fb, gb, f0b, g0b, sb, rcb) = _both(laue, P, scale, rho)
        print(f"rho {rho}: {len(P.obs['p12'])} detected, {len(P.model['m'])} model spots: workspace call {sa} "
              f"rc {rca}; scratch call {sb} rc {rcb}", flush=True)
        assert rca == rcb and sa["converged"] == sb["converged"]
        assert sa["n_iter"] == sb["n_iter"] and sa["err"] == sb["err"]
        assert torch.equal(fa, fb) and torch.equal(ga, gb)
        assert f0a == f0b and g0a == g0b


def test_noalloc_refuses_a_problem_beyond_its_scratch(gpu_lib):
    laue = gpu_lib
    lib = laue.require_native()
    cap = lib.laue_sinkhorn_noalloc_capacity()
    assert cap == 64 << 20
    p = ig.LEARNED
    geom = laue.geometry_from_preset(p)
    need = lib.laue_sinkhorn_workspace_size(laue.C.byref(geom), 900_000, 500_000, 0)
    assert need > cap
    # sizes only: the arrays are never touched because the call is refused first
    obs = laue.ObsSpots(torch.zeros(900_000, device="cuda"), torch.zeros(900_000, device="cuda"),
                        np.linspace(0, 900_000, geom.n_rot * geom.n_det + 1).astype(np.int64))
    model = laue.ModelSpots(500_000, geom.n_rot * geom.n_det)
    model.block_off[:] = np.linspace(0, 500_000, geom.n_rot * geom.n_det + 1).astype(np.int64)
    ot = laue.ot_params(1.0, p.distance, 9.0, 200_000.0)
    f = torch.zeros(900_000, device="cuda")
    g = torch.zeros(500_000, device="cuda")
    with pytest.raises(laue.LaueError) as ex:
        laue.laue_sinkhorn_noalloc(geom, obs, model, ot, f, g)
    assert ex.value.code == -3 and "bytes of scratch" in str(ex.value)
