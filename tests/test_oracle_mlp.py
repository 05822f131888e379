"""Pins of the oracle network: bfloat16 rounding, finite-difference
gradients, and that Adam training separates a learnable toy problem."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7                     # bfloat16 spacing at 1
    assert mlp.bf16(one) == one
    assert mlp.bf16(one + ulp / 2) == one               # tie -> even (1.0)
    assert mlp.bf16(one + 3 * ulp / 2) == one + 2 * ulp  # tie -> even mantissa
    assert mlp.bf16(one + 0.51 * ulp) == one + ulp
    assert mlp.bf16(-one - 0.49 * ulp) == -one
    x = np.random.default_rng(0).standard_normal(1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * 1.0001)
    assert np.array_equal(mlp.bf16(r), r)               # idempotent


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    p = mlp.init(16, 24, seed=2)
    x = rng.standard_normal((12, 16))
    y = (rng.uniform(size=12) < 0.4).astype(float)
    g, _ = mlp.backward(p, x, y, round_=False)
    h = 1e-6
    for k in p:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pm = {kk: vv.copy() for kk, vv in p.items()}
            pp[k].ravel()[idx] += h
            pm[k].ravel()[idx] -= h
            num = (mlp.loss(pp, x, y, False) - mlp.loss(pm, x, y, False)) / (2 * h)
            assert g[k].ravel()[idx] == pytest.approx(num, rel=1e-5, abs=1e-9)


def test_rounded_forward_close_to_exact():
    rng = np.random.default_rng(3)
    p = mlp.init(seed=4)
    x = rng.standard_normal((64, 16))
    pr, _ = mlp.forward(p, x, True)
    pe, _ = mlp.forward(p, x, False)
    assert np.max(np.abs(pr - pe)) < 2e-2


def test_adam_learns_toy_problem():
    rng = np.random.default_rng(5)
    p = mlp.init(16, 32, seed=6)
    x = rng.standard_normal((512, 16))
    y = (x[:, 0] + 0.5 * x[:, 1] > 0.3).astype(float)
    st = {}
    l0 = mlp.loss(p, x, y)
    for t in range(1, 151):
        g, _ = mlp.backward(p, x, y)
        p, st = mlp.adam(p, g, st, t, lr=1e-2)
    assert mlp.loss(p, x, y) < 0.5 * l0
    prob, _ = mlp.forward(p, x)
    assert np.mean((prob > 0.5) == (y > 0.5)) > 0.9
