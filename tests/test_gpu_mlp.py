"""GPU parity of the learned-proposal network against the oracle network:
forward probabilities, gradients of the BCE loss and one Adam step, with the
same bfloat16 rounding points on both sides."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _data(B=512, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, 16)).astype(np.float32)
    y = (x[:, 0] - 0.7 * x[:, 3] + 0.2 * rng.standard_normal(B) > 0.4).astype(np.float32)
    return x, y


def test_forward_matches_oracle(gpu_lib):
    laue = gpu_lib
    p = omlp.init(seed=3)
    net = laue.Mlp(params=laue.Mlp.pack(p))
    for B in (1, 37, 700, 70000):
        x, _ = _data(B, seed=B)
        pg = laue.laue_mlp_forward(net, torch.tensor(x, device="cuda")).cpu().numpy()
        po, _ = omlp.forward(p, x.astype(np.float64))
        assert np.max(np.abs(pg - po)) < 2e-3, B


def test_gradients_and_adam_match_oracle(gpu_lib):
    laue = gpu_lib
    p = omlp.init(seed=5)
    # a trained-like state so that gradients are not dominated by the init
    p["b1"] = np.random.default_rng(1).uniform(-0.1, 0.1, 256).astype(np.float32).astype(np.float64)
    net = laue.Mlp(params=laue.Mlp.pack(p))
    x, y = _data(1024, seed=7)
    gg, lg = laue.laue_mlp_backward(net, torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"))
    go, po = omlp.backward(p, x.astype(np.float64), y.astype(np.float64))
    assert lg == pytest.approx(omlp.loss(p, x.astype(np.float64), y.astype(np.float64)), rel=2e-3)
    gd = laue.Mlp.unpack(gg.cpu().numpy())
    for k in go:
        rel = np.linalg.norm(gd[k] - go[k]) / max(np.linalg.norm(go[k]), 1e-12)
        assert rel < 5e-3, (k, rel)
    # one Adam step from the same gradients
    ap = laue.adam_params(lr=1e-3)
    laue.laue_mlp_adam(net, gg, ap)
    pn, _ = omlp.adam(p, {k: gd[k] for k in gd}, {}, 1, lr=1e-3)
    got = laue.Mlp.unpack(net.params.cpu().numpy())
    for k in pn:
        assert np.max(np.abs(got[k] - pn[k])) < 1e-6 + 1e-6 * np.max(np.abs(pn[k]))


def test_training_reduces_loss(gpu_lib):
    laue = gpu_lib
    net = laue.Mlp(seed=11)
    x, y = _data(4096 * 4, seed=9)
    xt, yt = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
    tr = laue.MlpTrainer(net, 4096, laue.adam_params(lr=3e-3))
    losses = []
    for ep in range(30):
        for b in range(4):
            losses.append(tr.laue_mlp_train_step(xt[b * 4096:(b + 1) * 4096].contiguous(),
                                                 yt[b * 4096:(b + 1) * 4096].contiguous()))
    assert losses[-1] < 0.5 * losses[0]
    prob = laue.laue_mlp_forward(net, xt).cpu().numpy()
    assert np.mean((prob > 0.5) == (y > 0.5)) > 0.9
