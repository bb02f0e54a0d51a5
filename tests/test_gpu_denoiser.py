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


# (base width, edge): c = 8 runs every layer through the implicit GEMM; c = 32
# sends the two outer levels (32 and 64 channels on 16^3 and 8^3 grids)
# through the direct brick convolution
@pytest.fixture(scope="module", params=[(8, 16), (32, 16)], ids=["c8", "c32"])
def case(request):
    from oracle import denoiser as D
    rng = np.random.default_rng(8)
    c, n = request.param
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
    _, g_pert = _bf16_gradients(D, p, x, target, perturb=np.random.default_rng(9))
    return dict(D=D, c=c, n=n, shapes=shapes, p=p, x=x, target=target, loss=loss, g=g, y=y,
                g_bf=g_bf, g_pert=g_pert)


def _bf16(a, perturb=None):
    """Round to the nearest BF16 (ties to even), returned as float64.  With
    a generator, every value is first scaled by 1 + 2^-21 * N(0, 1): a
    relative disturbance below what FP32 accumulation of a few hundred terms
    leaves, which moves a value across a BF16 rounding boundary only when it
    lies within that distance of one."""
    a = np.asarray(a, dtype=np.float64)
    if perturb is not None:
        a = a * (1.0 + 2.0 ** -21 * perturb.standard_normal(a.shape))
    u = a.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_gradients(D, p, x, target, perturb=None):
    """The oracle's FP64 backward with every tensor that the GPU stores in
    BF16 (layer inputs, weights, ReLU outputs, transposed-conv outputs and the
    gradients passed between layers) rounded to BF16 where the GPU rounds it.
    Isolates the precision the kernels compute in from their arithmetic.
    With `perturb`, the roundings of computed values (not of the weights,
    which both sides convert identically) see a disturbance of FP32 size; the
    spread between the two runs is how far accumulation order alone can move
    each gradient."""
    from unittest import mock
    conv3, conv3_b, tconv2, tconv2_b, relu = (D.conv3, D.conv3_backward, D.tconv2,
                                              D.tconv2_backward, D.relu)

    def rb(a):
        return _bf16(a, perturb)

    def cb(xx, w, gy):
        gx, gw, gb = conv3_b(rb(xx), _bf16(w), rb(gy))
        return rb(gx), gw, gb

    def tb(xx, w, gy):
        gx, gw, gb = tconv2_b(rb(xx), _bf16(w), rb(gy))
        return rb(gx), gw, gb

    with mock.patch.multiple(D, conv3=lambda xx, w, b: conv3(rb(xx), _bf16(w), b),
                             tconv2=lambda xx, w, b: rb(tconv2(rb(xx), _bf16(w), b)),
                             conv3_backward=cb, tconv2_backward=tb,
                             relu=lambda z: rb(relu(z))):
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
    only by FP32 accumulation order, which flips a BF16 rounding wherever a
    value lies near a boundary.  On the few-voxel deep levels (4^3 and 2^3
    here) such flips, amplified through ReLU masks and pooling choices, move
    a gradient by several percent: the same emulation with an FP32-sized
    disturbance (spread s per tensor) measures this, and the bound is
    3 % + 3 s per tensor (s is below 1 % on the 16^3 and 8^3 levels).  The
    emulation itself stays within 20 % of the plain FP64 gradient and the GPU
    gradient points the same way (cosine > 0.97)."""
    net, inp, tgt = _net(eng, case)
    g, loss = net.gradients(inp, tgt)
    assert loss == pytest.approx(case["loss"], rel=3e-2)
    gd = _unflat(g.astype(np.float64), case["shapes"])
    errs, spreads, sizes = [], [], []
    for name, _ in case["shapes"]:
        ref = case["g"][name]
        ref_bf = case["g_bf"][name]
        got = gd[name]
        nr, nb = np.linalg.norm(ref), np.linalg.norm(ref_bf)
        if nr == 0:
            continue
        rel = np.linalg.norm(got - ref) / nr
        rel_bf = np.linalg.norm(got - ref_bf) / nb
        emu = np.linalg.norm(ref_bf - ref) / nr
        spread = np.linalg.norm(case["g_pert"][name] - ref_bf) / nb
        cos = float(np.dot(got.ravel(), ref.ravel()) / (np.linalg.norm(got) * nr + 1e-300))
        print(f"{name:10s} rel {rel:.4f} cos {cos:.5f} rel_vs_bf16_oracle {rel_bf:.4f} "
              f"spread {spread:.4f}")
        errs.append(rel_bf)
        spreads.append(spread)
        sizes.append(ref.size)
        assert rel_bf < 0.03 + 3.0 * spread, (name, rel_bf, spread)
        assert emu < 0.2 and cos > 0.97, (name, emu, cos)
    # parameter-count weighted means against the BF16-rounded oracle
    assert np.average(errs, weights=sizes) < 0.02 + 2.0 * np.average(spreads, weights=sizes)


def test_training_lowers_loss(eng, case):
    import torch
    net, inp, tgt = _net(eng, case)
    losses = []
    for i in range(40):
        lp = net.train_step(inp, tgt, 1e-3)
        torch.cuda.synchronize()
        losses.append(float(lp.sum().item()))
    assert losses[-1] < 0.5 * losses[0], losses[::10]


@pytest.fixture(scope="module")
def case64():
    """Base width 8 on a 64^3 volume: the four levels hold 64^3, 32^3, 16^3
    and 8^3 voxels, so no gradient rests on a few-voxel level."""
    from oracle import denoiser as D
    rng = np.random.default_rng(8)
    c, n = 8, 64
    shapes = D.param_shapes(c, 2)
    p = D.init_params(4, c=c)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    p["head.w"] = p["head.w"] * 10.0
    x = np.stack([rng.uniform(0, 1, (n, n, n)), rng.uniform(0.2, 1.8, (n, n, n))])
    target = x[0] + 0.1 * rng.standard_normal((n, n, n))
    print("[denoiser parity] FP64 oracle gradients at 64^3", flush=True)
    loss, g = D.loss_and_grad(p, x, target)
    print("[denoiser parity] BF16-emulated oracle gradients at 64^3", flush=True)
    _, g_bf = _bf16_gradients(D, p, x, target)
    return dict(D=D, c=c, n=n, shapes=shapes, p=p, x=x, target=target, loss=loss, g=g, g_bf=g_bf)


def test_gradients_match_oracle_flat_bound_at_64(eng, case64):
    """Every parameter gradient within 3 % (relative L2) of the oracle with
    BF16 rounding emulated where the GPU stores BF16, and pointing the same
    way as the plain FP64 gradient (cosine >= 0.998), on a volume whose
    deepest level still holds 8^3 voxels."""
    net, inp, tgt = _net(eng, case64)
    g, loss = net.gradients(inp, tgt)
    assert loss == pytest.approx(case64["loss"], rel=1e-2)
    gd = _unflat(g.astype(np.float64), case64["shapes"])
    worst = 0.0
    for name, _ in case64["shapes"]:
        ref, ref_bf, got = case64["g"][name], case64["g_bf"][name], gd[name]
        nr = np.linalg.norm(ref)
        if nr == 0:
            continue
        rel_bf = np.linalg.norm(got - ref_bf) / np.linalg.norm(ref_bf)
        cos = float(np.dot(got.ravel(), ref.ravel()) / (np.linalg.norm(got) * nr))
        worst = max(worst, rel_bf)
        assert rel_bf < 0.03, (name, rel_bf)
        assert cos >= 0.998, (name, cos)
    print(f"[denoiser parity] 64^3: worst relative L2 against the BF16-emulated oracle "
          f"{worst:.4f}", flush=True)
