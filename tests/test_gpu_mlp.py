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


def test_gradients_elementwise_at_training_batch(gpu_lib):
    """Every gradient element at batch 4096.  Both sides round the same values
    to bfloat16; what remains is FP32 accumulation (about 1e-7 relative on each
    product) and the rare bfloat16 rounding it flips (one activation moved by
    one bfloat16 ulp, 2^-8 relative, in one of 4096 terms of a sum).  Either is
    far below 1e-3 of the tensor's largest element plus 1e-3 relative."""
    laue = gpu_lib
    p = omlp.init(seed=6)
    p["b1"] = np.random.default_rng(2).uniform(-0.1, 0.1, 256).astype(np.float32).astype(np.float64)
    p["b2"] = np.random.default_rng(3).uniform(-0.05, 0.05, 256).astype(np.float32).astype(np.float64)
    net = laue.Mlp(params=laue.Mlp.pack(p))
    x, y = _data(4096, seed=8)
    gg, _ = laue.laue_mlp_backward(net, torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"))
    go, _ = omlp.backward(p, x.astype(np.float64), y.astype(np.float64))
    gd = laue.Mlp.unpack(gg.cpu().numpy())
    for k in go:
        bound = 1e-3 * np.max(np.abs(go[k])) + 1e-3 * np.abs(go[k])
        err = np.abs(gd[k] - go[k])
        assert np.all(err <= bound), (k, float(np.max(err / bound)))


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


def _epoch_order(n, seed, epoch):
    """The documented epoch order, from the oracle's Philox: example i gets the
    key of counter (i, epoch, 0, 8); increasing key, ties by index."""
    from oracle import philox
    i = np.arange(n, dtype=np.uint64)
    keys = philox.key64(i, np.uint64(epoch), np.uint64(0), np.uint64(8), seed)
    return np.lexsort((np.arange(n), keys))


@pytest.mark.parametrize("n,batch", [(1636, 512), (4096, 4096), (70000, 4096)])
def test_epoch_is_the_documented_order_of_train_steps(gpu_lib, n, batch):
    """laue_mlp_train_epoch equals laue_mlp_train_step over the batches of the
    documented seeded order (ragged tail left out), bit for bit, two epochs."""
    laue = gpu_lib
    x, y = _data(n, seed=n)
    xt, yt = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
    a, b = laue.Mlp(seed=2), laue.Mlp(seed=2)
    ap = laue.adam_params(lr=2e-3)
    tr = laue.MlpTrainer(b, batch, ap)
    seed = 0x1234_5678_9ABC
    for ep in range(2):
        la = laue.laue_mlp_train_epoch(a, xt, yt, batch, seed, ep, ap)
        order = torch.tensor(_epoch_order(n, seed, ep), device="cuda")
        nb = n // batch
        lb = [tr.laue_mlp_train_step(xt[order[k * batch:(k + 1) * batch]].contiguous(),
                                     yt[order[k * batch:(k + 1) * batch]].contiguous()) for k in range(nb)]
        assert la == pytest.approx(float(np.mean(lb)), rel=1e-12)
        assert torch.equal(a.params, b.params), ep
        assert torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
    # another epoch index or seed draws another order
    o0, o1, o2 = _epoch_order(n, seed, 0), _epoch_order(n, seed, 1), _epoch_order(n, seed + 1, 0)
    assert not np.array_equal(o0, o1) and not np.array_equal(o0, o2)


def test_epoch_rejects_bad_sizes(gpu_lib):
    laue = gpu_lib
    x, y = _data(100, seed=1)
    xt, yt = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
    net = laue.Mlp(seed=1)
    ap = laue.adam_params()
    before = net.params.clone()
    for batch in (128, 24):  # more than n; not a multiple of 16
        with pytest.raises(laue.LaueError):
            laue.laue_mlp_train_epoch(net, xt, yt, batch, 0, 0, ap)
    assert torch.equal(net.params, before)
