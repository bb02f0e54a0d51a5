"""GPU denoiser kernels (BF16 MFMA, FP32 accumulation) against the FP64
oracle: forward prediction, loss and every parameter gradient of a small
network, at tolerances that allow for BF16 activations and weights; and a
training run that lowers the loss."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _flat(p, shapes):
    return np.concatenate([p[n].ravel() for n, _ in shapes])


def _unflat(v, shapes):
    out, i = {}, 0
    for n, s in shapes:
        k = int(np.prod(s))
        out[n] = v[i:i + k].reshape(s)
        i += k
    return out


@pytest.fixture(scope="module")
def case():
    from oracle import denoiser as D
    rng = np.random.default_rng(8)
    c, n = 8, 16
    shapes = D.param_shapes(c, 2)
    p = D.init_params(4, c=c)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    p["head.w"] = p["head.w"] * 10.0
    x = np.stack([rng.uniform(0, 1, (n, n, n)), rng.uniform(0.2, 1.8, (n, n, n))])
    target = x[0] + 0.1 * rng.standard_normal((n, n, n))
    loss, g = D.loss_and_grad(p, x, target)
    y, _ = D.forward(p, x)
    return dict(D=D, c=c, n=n, shapes=shapes, p=p, x=x, target=target, loss=loss, g=g, y=y)


def _net(eng, case):
    import torch
    net = eng.UNet(case["c"], case["n"], case["n"], case["n"])
    assert net.n_params == sum(int(np.prod(s)) for _, s in case["shapes"])
    net.set_params(_flat(case["p"], case["shapes"]).astype(np.float32))
    inp = torch.as_tensor(case["x"].astype(np.float32), device="cuda").contiguous()
    tgt = torch.as_tensor(case["target"].astype(np.float32), device="cuda").contiguous()
    return net, inp, tgt


def test_forward_matches_oracle(eng, case):
    import torch
    net, inp, tgt = _net(eng, case)
    y = net.forward(inp)
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    ref = case["y"]
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert err < 1e-2, err


def test_gradients_match_oracle(eng, case):
    net, inp, tgt = _net(eng, case)
    g, loss = net.gradients(inp, tgt)
    assert loss == pytest.approx(case["loss"], rel=3e-2)
    gd = _unflat(g.astype(np.float64), case["shapes"])
    for name, _ in case["shapes"]:
        ref = case["g"][name]
        got = gd[name]
        nr = np.linalg.norm(ref)
        if nr == 0:
            continue
        rel = np.linalg.norm(got - ref) / nr
        cos = float(np.dot(got.ravel(), ref.ravel()) / (np.linalg.norm(got) * nr + 1e-300))
        assert rel < 5e-2 and cos > 0.998, (name, rel, cos)


def test_training_lowers_loss(eng, case):
    import torch
    net, inp, tgt = _net(eng, case)
    losses = []
    for i in range(40):
        lp = net.train_step(inp, tgt, 1e-3)
        torch.cuda.synchronize()
        losses.append(float(lp.sum().item()))
    assert losses[-1] < 0.5 * losses[0], losses[::10]
