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
    _, g_bf = _bf16_gradients(D, p, x, target)
    return dict(D=D, c=c, n=n, shapes=shapes, p=p, x=x, target=target, loss=loss, g=g, y=y,
                g_bf=g_bf)


def _bf16(a):
    """Round to the nearest BF16 (ties to even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_gradients(D, p, x, target):
    """The oracle's FP64 backward with every tensor that the GPU stores in
    BF16 (layer inputs, weights, ReLU outputs, transposed-conv outputs and the
    gradients passed between layers) rounded to BF16 where the GPU rounds it.
    Isolates the precision the kernels compute in from their arithmetic."""
    from unittest import mock
    conv3, conv3_b, tconv2, tconv2_b, relu = (D.conv3, D.conv3_backward, D.tconv2,
                                              D.tconv2_backward, D.relu)

    def cb(xx, w, gy):
        gx, gw, gb = conv3_b(_bf16(xx), _bf16(w), _bf16(gy))
        return _bf16(gx), gw, gb

    def tb(xx, w, gy):
        gx, gw, gb = tconv2_b(_bf16(xx), _bf16(w), _bf16(gy))
        return _bf16(gx), gw, gb

    with mock.patch.multiple(D, conv3=lambda xx, w, b: conv3(_bf16(xx), _bf16(w), b),
                             tconv2=lambda xx, w, b: _bf16(tconv2(_bf16(xx), _bf16(w), b)),
                             conv3_backward=cb, tconv2_backward=tb,
                             relu=lambda z: _bf16(relu(z))):
        return D.loss_and_grad(p, x, target)


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
    """Every parameter gradient against the oracle.  Against the FP64 oracle
    with BF16 rounding applied where the GPU stores BF16, the kernels differ
    only by FP32 accumulation order: relative L2 error < 3 % per tensor.
    Against the plain FP64 oracle the BF16 rounding itself (up to ~13 % on
    the deepest, 2^3-voxel layers of this 16^3 case, measured with the same
    emulation) bounds the error: < 20 % per tensor and cosine > 0.985."""
    net, inp, tgt = _net(eng, case)
    g, loss = net.gradients(inp, tgt)
    assert loss == pytest.approx(case["loss"], rel=3e-2)
    gd = _unflat(g.astype(np.float64), case["shapes"])
    errs, sizes = [], []
    for name, _ in case["shapes"]:
        ref = case["g"][name]
        ref_bf = case["g_bf"][name]
        got = gd[name]
        nr = np.linalg.norm(ref)
        if nr == 0:
            continue
        rel = np.linalg.norm(got - ref) / nr
        rel_bf = np.linalg.norm(got - ref_bf) / np.linalg.norm(ref_bf)
        cos = float(np.dot(got.ravel(), ref.ravel()) / (np.linalg.norm(got) * nr + 1e-300))
        print(f"{name:10s} rel {rel:.4f} cos {cos:.5f} rel_vs_bf16_oracle {rel_bf:.4f}")
        errs.append(rel_bf)
        sizes.append(ref.size)
        assert rel_bf < 0.03, (name, rel_bf)
        assert rel < 0.2 and cos > 0.985, (name, rel, cos)
    # parameter-count weighted mean against the BF16-rounded oracle
    assert np.average(errs, weights=sizes) < 0.02


def test_training_lowers_loss(eng, case):
    import torch
    net, inp, tgt = _net(eng, case)
    losses = []
    for i in range(40):
        lp = net.train_step(inp, tgt, 1e-3)
        torch.cuda.synchronize()
        losses.append(float(lp.sum().item()))
    assert losses[-1] < 0.5 * losses[0], losses[::10]
