"""FP64 numpy reference of the learned 3D dose denoiser (a small U-Net).

TEST INFRASTRUCTURE ONLY (tests, smoke, benchmark baseline).  Shares no code
with the GPU kernels.  The paper has no denoiser; the network follows the
documented reading:

  * input: 2 channels (dose / its maximum, density), D^3 voxels, D divisible by 8
  * 4 resolution levels with c, 2c, 4c, 8c channels (c = base width);
    each level: two 3x3x3 convolutions (zero padding 1) each followed by ReLU
  * down: 2x2x2 max pooling; up: 2x2x2 stride-2 transposed convolution,
    concatenated with the encoder output of the same level (skip first)
  * head: 1x1x1 convolution to one channel, plus the scaled input dose
    (residual), loss = mean squared error against the scaled target

Activations are [C, D, H, W] arrays; conv weights [C_out, C_in, 3, 3, 3];
transposed-conv weights [C_in, C_out, 2, 2, 2]; the head [1, c].
Backward passes are written out by hand.  Pins: torch CPU float64 ops for
each layer, central finite differences for the whole network.
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# Layers
# --------------------------------------------------------------------------
def conv3(x, w, b):
    """3x3x3 convolution, stride 1, zero padding 1 (cross-correlation)."""
    c_in, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    y = np.broadcast_to(b[:, None, None, None], (w.shape[0], D, H, W)).copy()
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                y += np.einsum("oc,czyx->ozyx", w[:, :, dz, dy, dx],
                               xp[:, dz:dz + D, dy:dy + H, dx:dx + W])
    return y


def conv3_backward(x, w, gy):
    """Gradients of conv3 with respect to x, w and b."""
    c_in, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                sl = (slice(None), slice(dz, dz + D), slice(dy, dy + H), slice(dx, dx + W))
                gxp[sl] += np.einsum("oc,ozyx->czyx", w[:, :, dz, dy, dx], gy)
                gw[:, :, dz, dy, dx] = np.einsum("ozyx,czyx->oc", gy, xp[sl])
    return gxp[:, 1:-1, 1:-1, 1:-1], gw, gy.sum(axis=(1, 2, 3))


def relu(x):
    return np.maximum(x, 0.0)


def relu_backward(x, gy):
    return gy * (x > 0.0)


def maxpool2(x):
    """2x2x2 max pooling; returns the output and the in-block index of the
    maximum (first maximum in z, y, x order)."""
    c, D, H, W = x.shape
    blk = x.reshape(c, D // 2, 2, H // 2, 2, W // 2, 2).transpose(0, 1, 3, 5, 2, 4, 6)
    blk = blk.reshape(c, D // 2, H // 2, W // 2, 8)
    idx = blk.argmax(axis=-1)
    return np.take_along_axis(blk, idx[..., None], axis=-1)[..., 0], idx


def maxpool2_backward(idx, gy, shape):
    c, D, H, W = shape
    g8 = np.zeros(gy.shape + (8,))
    np.put_along_axis(g8, idx[..., None], gy[..., None], axis=-1)
    g = g8.reshape(c, D // 2, H // 2, W // 2, 2, 2, 2).transpose(0, 1, 4, 2, 5, 3, 6)
    return g.reshape(shape)


def tconv2(x, w, b):
    """2x2x2 transposed convolution with stride 2: each input voxel writes
    one 2x2x2 output block; w is [C_in, C_out, 2, 2, 2]."""
    c_in, D, H, W = x.shape
    c_out = w.shape[1]
    y = np.einsum("czyx,coabd->ozaybxd", x, w).reshape(c_out, 2 * D, 2 * H, 2 * W)
    return y + b[:, None, None, None]


def tconv2_backward(x, w, gy):
    c_in, D, H, W = x.shape
    c_out = w.shape[1]
    g = gy.reshape(c_out, D, 2, H, 2, W, 2)
    gx = np.einsum("ozaybxd,coabd->czyx", g, w)
    gw = np.einsum("czyx,ozaybxd->coabd", x, g)
    return gx, gw, gy.sum(axis=(1, 2, 3))


# --------------------------------------------------------------------------
# Network
# --------------------------------------------------------------------------
LEVELS = 4


def param_shapes(c=32, c_in=2):
    """Ordered parameter list: (name, shape)."""
    out = []
    widths = [c * 2 ** k for k in range(LEVELS)]
    prev = c_in
    for k, wk in enumerate(widths):
        out += [(f"enc{k}a.w", (wk, prev, 3, 3, 3)), (f"enc{k}a.b", (wk,)),
                (f"enc{k}b.w", (wk, wk, 3, 3, 3)), (f"enc{k}b.b", (wk,))]
        prev = wk
    for k in range(LEVELS - 2, -1, -1):
        wk = widths[k]
        out += [(f"up{k}.w", (widths[k + 1], wk, 2, 2, 2)), (f"up{k}.b", (wk,)),
                (f"dec{k}a.w", (wk, 2 * wk, 3, 3, 3)), (f"dec{k}a.b", (wk,)),
                (f"dec{k}b.w", (wk, wk, 3, 3, 3)), (f"dec{k}b.b", (wk,))]
    out += [("head.w", (1, c)), ("head.b", (1,))]
    return out


def init_params(seed, c=32, c_in=2):
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in param_shapes(c, c_in):
        if name.endswith(".b"):
            p[name] = np.zeros(shape)
        elif name.startswith("up"):
            fan_in = shape[0]          # each output voxel sees C_in inputs
            p[name] = rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)
        elif name == "head.w":
            p[name] = rng.standard_normal(shape) * np.sqrt(1.0 / shape[1]) * 0.1
        else:
            fan_in = shape[1] * 27
            p[name] = rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)
    return p


def forward(p, x):
    """x: [2, D, H, W] (scaled dose, density).  Returns (prediction [D,H,W], cache)."""
    cache = {"x": x}
    h = x
    skips = []
    for k in range(LEVELS):
        if k > 0:
            h, idx = maxpool2(h)
            cache[f"pool{k}"] = (idx, skips[-1].shape)
        za = conv3(h, p[f"enc{k}a.w"], p[f"enc{k}a.b"])
        ha = relu(za)
        zb = conv3(ha, p[f"enc{k}b.w"], p[f"enc{k}b.b"])
        hb = relu(zb)
        cache[f"enc{k}"] = (h, za, ha, zb)
        h = hb
        skips.append(hb)
    for k in range(LEVELS - 2, -1, -1):
        u = tconv2(h, p[f"up{k}.w"], p[f"up{k}.b"])
        cat = np.concatenate([skips[k], u], axis=0)
        za = conv3(cat, p[f"dec{k}a.w"], p[f"dec{k}a.b"])
        ha = relu(za)
        zb = conv3(ha, p[f"dec{k}b.w"], p[f"dec{k}b.b"])
        hb = relu(zb)
        cache[f"dec{k}"] = (h, cat, za, ha, zb)
        h = hb
    y = np.einsum("c,czyx->zyx", p["head.w"][0], h) + p["head.b"][0] + x[0]
    cache["head"] = h
    return y, cache


def loss_and_grad(p, x, target):
    """MSE loss and the gradient of every parameter (hand-written backward)."""
    y, cache = forward(p, x)
    n = y.size
    loss = float(np.mean((y - target) ** 2))
    gy = 2.0 * (y - target) / n
    g = {}
    h = cache["head"]
    g["head.w"] = np.einsum("zyx,czyx->c", gy, h)[None, :]
    g["head.b"] = np.array([gy.sum()])
    gh = p["head.w"][0][:, None, None, None] * gy[None]
    skip_grads = {}
    for k in range(LEVELS - 1):
        h_in, cat, za, ha, zb = cache[f"dec{k}"]
        gzb = relu_backward(zb, gh)
        gha, g[f"dec{k}b.w"], g[f"dec{k}b.b"] = conv3_backward(ha, p[f"dec{k}b.w"], gzb)
        gza = relu_backward(za, gha)
        gcat, g[f"dec{k}a.w"], g[f"dec{k}a.b"] = conv3_backward(cat, p[f"dec{k}a.w"], gza)
        ck = cache[f"enc{k}"][3].shape[0]
        skip_grads[k] = gcat[:ck]
        gu = gcat[ck:]
        gh, g[f"up{k}.w"], g[f"up{k}.b"] = tconv2_backward(h_in, p[f"up{k}.w"], gu)
    for k in range(LEVELS - 1, -1, -1):
        h_in, za, ha, zb = cache[f"enc{k}"]
        if k in skip_grads:
            gh = gh + skip_grads[k]
        gzb = relu_backward(zb, gh)
        gha, g[f"enc{k}b.w"], g[f"enc{k}b.b"] = conv3_backward(ha, p[f"enc{k}b.w"], gzb)
        gza = relu_backward(za, gha)
        gh, g[f"enc{k}a.w"], g[f"enc{k}a.b"] = conv3_backward(h_in, p[f"enc{k}a.w"], gza)
        if k > 0:
            idx, shape = cache[f"pool{k}"]
            gh = maxpool2_backward(idx, gh, shape)
    return loss, g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015) in place."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for k in p:
        m = state.setdefault("m" + k, np.zeros_like(p[k]))
        v = state.setdefault("v" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


# --------------------------------------------------------------------------
# Evaluation metrics (Eq. 10 RMS as % of the reference maximum; gamma index)
# --------------------------------------------------------------------------
def rms_percent(d, ref, mask=None):
    """Eq. (10): RMS difference as a percentage of the reference maximum."""
    diff = (d - ref) if mask is None else (d - ref)[mask]
    return 100.0 * float(np.sqrt(np.mean(diff ** 2))) / float(ref.max())


def gamma_pass_rate(d, ref, vox, dd=0.02, dta=0.2, cutoff=0.1, search=0.4, sub=2):
    """Global gamma (dose difference dd of the reference maximum, distance to
    agreement dta in cm) over reference voxels above cutoff * max.  The
    evaluated dose is searched within `search` cm on a grid of 1/sub voxel
    steps, by trilinear interpolation."""
    from scipy import ndimage
    dmax = ref.max()
    step = [v / sub for v in vox]
    r = [int(np.ceil(search / s)) for s in step]
    best = np.full(ref.shape, np.inf)
    for kz in range(-r[0], r[0] + 1):
        for ky in range(-r[1], r[1] + 1):
            for kx in range(-r[2], r[2] + 1):
                dist2 = (kz * step[0]) ** 2 + (ky * step[1]) ** 2 + (kx * step[2]) ** 2
                if dist2 > search ** 2:
                    continue
                sh = ndimage.shift(d, (-kz / sub, -ky / sub, -kx / sub), order=1, mode="nearest")
                g2 = ((sh - ref) / (dd * dmax)) ** 2 + dist2 / dta ** 2
                np.minimum(best, g2, out=best)
    sel = ref > cutoff * dmax
    return float(np.mean(best[sel] <= 1.0))
