"""Seeded initial weights of the denoiser in the flat layout of psl.h
(He-normal convolutions, zero biases, a small head)."""
import numpy as np


def layer_shapes(c=32, c_in=2, levels=4):
    """(name, shape) in the order of the flat parameter array."""
    out = []
    widths = [c * 2 ** k for k in range(levels)]
    prev = c_in
    for k, wk in enumerate(widths):
        out += [(f"enc{k}a.w", (wk, prev, 3, 3, 3)), (f"enc{k}a.b", (wk,)),
                (f"enc{k}b.w", (wk, wk, 3, 3, 3)), (f"enc{k}b.b", (wk,))]
        prev = wk
    for k in range(levels - 2, -1, -1):
        wk = widths[k]
        out += [(f"up{k}.w", (widths[k + 1], wk, 2, 2, 2)), (f"up{k}.b", (wk,)),
                (f"dec{k}a.w", (wk, 2 * wk, 3, 3, 3)), (f"dec{k}a.b", (wk,)),
                (f"dec{k}b.w", (wk, wk, 3, 3, 3)), (f"dec{k}b.b", (wk,))]
    out += [("head.w", (c,)), ("head.b", (1,))]
    return out


def init_params(seed, c, n_expected=None):
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in layer_shapes(c):
        if name.endswith(".b"):
            parts.append(np.zeros(shape))
        elif name.startswith("up"):
            parts.append(rng.standard_normal(shape) * np.sqrt(2.0 / shape[0]))
        elif name == "head.w":
            parts.append(rng.standard_normal(shape) * 0.1 / np.sqrt(shape[0]))
        else:
            parts.append(rng.standard_normal(shape) * np.sqrt(2.0 / (shape[1] * 27)))
    flat = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
    if n_expected is not None:
        assert flat.size == n_expected, (flat.size, n_expected)
    return flat
