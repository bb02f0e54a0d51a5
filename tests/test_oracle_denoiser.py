"""Pins of the FP64 denoiser oracle: every layer against torch CPU float64
operations (an independent library), the hand-written backward against
torch autograd and against central finite differences of the whole network,
and the evaluation metrics on hand-built cases."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import denoiser as D


def _t(a, grad=False):
    return torch.tensor(a, dtype=torch.float64, requires_grad=grad)


def test_conv3_forward_and_backward_match_torch():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 6, 5, 4))
    w = rng.standard_normal((5, 3, 3, 3, 3))
    b = rng.standard_normal(5)
    y = D.conv3(x, w, b)
    tx, tw, tb = _t(x, True), _t(w, True), _t(b, True)
    ty = F.conv3d(tx[None], tw, tb, padding=1)[0]
    assert np.allclose(y, ty.detach().numpy(), rtol=1e-12, atol=1e-12)
    gy = rng.standard_normal(y.shape)
    ty.backward(_t(gy))
    gx, gw, gb = D.conv3_backward(x, w, gy)
    assert np.allclose(gx, tx.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(gw, tw.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(gb, tb.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_pool_and_transposed_conv_match_torch():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 4, 6, 2))
    y, idx = D.maxpool2(x)
    tx = _t(x, True)
    ty = F.max_pool3d(tx[None], 2)[0]
    assert np.array_equal(y, ty.detach().numpy())
    gy = rng.standard_normal(y.shape)
    ty.backward(_t(gy))
    assert np.allclose(D.maxpool2_backward(idx, gy, x.shape), tx.grad.numpy())
    w = rng.standard_normal((3, 4, 2, 2, 2))
    b = rng.standard_normal(4)
    y = D.tconv2(x, w, b)
    tx, tw, tb = _t(x, True), _t(w, True), _t(b, True)
    ty = F.conv_transpose3d(tx[None], tw, tb, stride=2)[0]
    assert np.allclose(y, ty.detach().numpy(), rtol=1e-12, atol=1e-12)
    gy = rng.standard_normal(y.shape)
    ty.backward(_t(gy))
    gx, gw, gb = D.tconv2_backward(x, w, gy)
    assert np.allclose(gx, tx.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(gw, tw.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(gb, tb.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = D.init_params(3, c=2)
    for k in p:                                  # non-zero biases exercise db paths
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    x = rng.uniform(0, 1, (2, 8, 8, 8))
    target = rng.uniform(0, 1, (8, 8, 8))
    loss, g = D.loss_and_grad(p, x, target)
    h = 1e-6
    for name in ("enc0a.w", "enc3b.w", "up2.w", "up0.b", "dec1a.w", "dec0b.b", "head.w"):
        flat = p[name].reshape(-1)
        for j in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[j]
            flat[j] = old + h
            lp, _ = D.forward(p, x)
            flat[j] = old - h
            lm, _ = D.forward(p, x)
            flat[j] = old
            fd = (np.mean((lp - target) ** 2) - np.mean((lm - target) ** 2)) / (2 * h)
            an = g[name].reshape(-1)[j]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-10), (name, j)


def test_param_count_of_the_workload_network():
    n = sum(int(np.prod(s)) for _, s in D.param_shapes(32, 2))
    assert 5.5e6 < n < 6.0e6


def test_adam_moves_against_gradient():
    p = {"w": np.array([1.0, -2.0])}
    g = {"w": np.array([0.5, -0.5])}
    st = {}
    D.adam_step(p, g, st, lr=0.1)
    assert np.allclose(p["w"], [0.9, -1.9])


def test_gamma_hand_built_cases():
    z = np.arange(40) * 0.25
    prof = 1.0 / (1.0 + np.exp(-(z - 5.0) / 0.3))          # a penumbra along z
    ref = np.broadcast_to(prof[:, None, None], (40, 8, 8)).copy()
    shifted = np.broadcast_to((1.0 / (1.0 + np.exp(-(z - 5.1) / 0.3)))[:, None, None],
                              (40, 8, 8)).copy()           # 1 mm shift
    # a 1 mm shift passes everywhere when the search grid resolves 0.5 mm
    assert D.gamma_pass_rate(shifted, ref, (0.25, 0.25, 0.25), sub=5) == 1.0
    scaled = ref * 1.03                                    # 3% everywhere
    flat = ref > 0.67 * ref.max()
    assert D.gamma_pass_rate(scaled, ref, (0.25, 0.25, 0.25)) < 1.0
    assert D.rms_percent(scaled, ref, flat) == pytest.approx(
        100 * np.sqrt(np.mean((0.03 * ref[flat]) ** 2)) / ref.max())
