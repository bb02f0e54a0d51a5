"""Denoiser pipeline: training pairs from the engine, training on the GPU
through psl_unet_*, and evaluation of denoised against plain doses.

Cases (seeded): a heterogeneous water / lung / bone phantom resampled to
n^3 voxels, one field with jaw sizes U[3, 15] cm at a gantry angle
U[0, 360) degrees.  The network input is (low-history dose / its maximum,
density); the target is the high-history dose on the same scale.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

from . import workloads as wl


# history counts of the evaluated plain / denoised doses
EVAL_COUNTS = (1e6, 3e6, 1e7, 3e7, 1e8)
RMS_TARGETS = (2.0, 1.0, 0.6)   # stated RMS errors, % of Dmax


def case_geometry(seed, n=128, vox=0.25):
    rng = np.random.Generator(np.random.PCG64([int(seed), 4242]))
    ph = wl.hetero_phantom(seed, nx=n, ny=n, nz=n, vox=vox)
    fx, fy = rng.uniform(3.0, 15.0, size=2)
    g = float(rng.uniform(0.0, 360.0))
    beam = wl.Beam(-fx / 2, fx / 2, -fy / 2, fy / 2, g, 0.0, (0.0, 0.0, 0.0))
    return ph, beam


class DoseEngine:
    """Plain engine runs for one phantom and beam (native runtime)."""

    def __init__(self, model_src, phantom, beam, seed):
        from . import engine as eng
        self.eng = eng
        self.model = eng.Model(model_src)
        self.phantom = eng.Phantom(phantom)
        self.beam = beam
        self.seed = seed
        self.prm = eng.transport_params()

    def dose(self, n_hist, n_rep=4, seed_offset=0, max_batch=1 << 20):
        """Dose and standard error (Gy per model particle, torch on the GPU)."""
        import torch
        eng = self.eng
        per = max(1, n_hist // n_rep)
        plan = eng.Plan(self.model, [self.beam], per, n_replica=n_rep)
        tally = eng.Tally(self.phantom)
        eng.run_plan(plan, self.phantom, tally, self.prm,
                     eng.run_opts(min(max_batch, max(4096, per)), 24, use_graph=False,
                                  seed=self.seed * 1000003 + seed_offset))
        d, s = tally.finalize(plan)
        torch.cuda.synchronize()
        return d.float(), s.float()


def rms_percent(d, ref, mask=None):
    """RMS difference as a percentage of the reference maximum (Eq. 10)."""
    diff = d - ref
    if mask is not None:
        diff = diff[mask]
    return 100.0 * float(np.sqrt(np.mean(diff.astype(np.float64) ** 2))) / float(ref.max())


def gamma_pass_rate(d, ref, vox, dd=0.02, dta=0.2, cutoff=0.1, search=0.4, sub=2):
    """Global gamma pass rate: dose criterion dd of the reference maximum,
    distance criterion dta (cm), over reference voxels above cutoff * max;
    the evaluated dose is trilinearly shifted on a 1/sub-voxel grid within
    `search` cm and the smallest gamma^2 kept."""
    import torch
    dev = "cuda" if torch.cuda.is_available() else "cpu"
    dt = torch.as_tensor(d, dtype=torch.float32, device=dev)[None, None]
    rt = torch.as_tensor(ref, dtype=torch.float32, device=dev)
    dmax = float(rt.max())
    D, H, W = ref.shape
    best = torch.full_like(rt, float("inf"))
    zs = torch.linspace(-1, 1, D, device=dev)
    ys = torch.linspace(-1, 1, H, device=dev)
    xs = torch.linspace(-1, 1, W, device=dev)
    gz, gy, gx = torch.meshgrid(zs, ys, xs, indexing="ij")
    step = [v / sub for v in vox]
    r = [int(math.ceil(search / s)) for s in step]
    for kz in range(-r[0], r[0] + 1):
        for ky in range(-r[1], r[1] + 1):
            for kx in range(-r[2], r[2] + 1):
                dist2 = (kz * step[0]) ** 2 + (ky * step[1]) ** 2 + (kx * step[2]) ** 2
                if dist2 > search ** 2:
                    continue
                # sample d at (p + offset): normalised grid coordinates
                oz = kz / sub * 2.0 / max(D - 1, 1)
                oy = ky / sub * 2.0 / max(H - 1, 1)
                ox = kx / sub * 2.0 / max(W - 1, 1)
                grid = torch.stack([gx + ox, gy + oy, gz + oz], dim=-1)[None]
                sh = torch.nn.functional.grid_sample(dt, grid, mode="bilinear",
                                                     padding_mode="border",
                                                     align_corners=True)[0, 0]
                g2 = ((sh - rt) / (dd * dmax)) ** 2 + dist2 / dta ** 2
                best = torch.minimum(best, g2)
    sel = rt > cutoff * dmax
    return float((best[sel] <= 1.0).float().mean())


def sigma_rel(d, s, frac=0.5):
    """RMS of sigma/D over voxels with D above frac * Dmax."""
    sel = d > frac * d.max()
    return float(np.sqrt(np.mean((s[sel] / d[sel]) ** 2)))


def make_pairs(seeds, n_low, n_high, model_src, n=128, log=print):
    """Training / evaluation cases: (input [2,n,n,n] float32, target [n,n,n],
    reference scale) with doses divided by the low-history dose maximum."""
    import torch
    out = []
    for i, s in enumerate(seeds):
        ph, beam = case_geometry(s, n)
        E = DoseEngine(model_src, ph, beam, s)
        lo, _ = E.dose(n_low, n_rep=1, seed_offset=1)
        hi, _ = E.dose(n_high, n_rep=1, seed_offset=2)
        scale = float(lo.max())
        inp = torch.stack([lo / scale, torch.as_tensor(ph.density, device="cuda")]).contiguous()
        out.append((inp, (hi / scale).contiguous(), scale))
        if (i + 1) % 10 == 0:
            log(f"[denoise] case {i + 1}/{len(seeds)}")
    return out


def train(net, pairs, epochs, lr, log=print, lr_decay=0.5):
    import torch
    rng = np.random.default_rng(0)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tot = 0.0
        rate = lr * (lr_decay ** (ep / max(1, epochs - 1)))
        for i in order:
            inp, tgt, _ = pairs[i]
            lp = net.train_step(inp, tgt, rate)
            tot += float(lp.sum())
        hist.append(tot / len(pairs))
        log(f"[denoise] epoch {ep + 1}/{epochs} mean loss {hist[-1]:.4e}")
    torch.cuda.synchronize()
    return hist


def unet_flops(c, n, levels=4):
    """Dense FP operations of one forward pass (a multiply-add counts 2) of the
    U-Net at base width c on an n^3 volume: 3x3x3 convolutions, 2x2x2
    transposed convolutions and the 1x1x1 head."""
    from .unet_init import layer_shapes
    f = 0.0
    for name, shape in layer_shapes(c, levels=levels):
        if not name.endswith(".w"):
            continue
        if name == "head.w":
            f += 2.0 * c * n ** 3
            continue
        lvl = int(name[3]) if name.startswith(("enc", "dec")) else int(name[2])
        p = (n >> lvl) ** 3                       # output voxels of the layer
        if name.startswith("up"):
            f += 2.0 * shape[0] * shape[1] * 8 * (n >> (lvl + 1)) ** 3
        else:
            f += 2.0 * shape[0] * shape[1] * 27 * p
    return f


def bench_unet(width=32, n=128, iters=10, log=print):
    """Forward and training-step time of the U-Net on an n^3 volume and the
    MFMA rate they reach (BF16 dense peak 2.5 PFLOP/s).  A training step is
    forward + backward (input-gradient and weight-gradient GEMMs, 2x the
    forward) + Adam."""
    import torch
    from . import engine as eng
    from .unet_init import init_params
    net = eng.UNet(width, n, n, n)
    net.set_params(init_params(7, width, net.n_params))
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    inp = torch.rand((2, n, n, n), generator=g, device="cuda")
    tgt = torch.rand((n, n, n), generator=g, device="cuda")
    for _ in range(2):
        net.forward(inp)
        net.train_step(inp, tgt, 1e-4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        net.forward(inp)
    e1.record()
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1) / iters
    e0.record()
    for _ in range(iters):
        net.train_step(inp, tgt, 1e-4)
    e1.record()
    torch.cuda.synchronize()
    t_train = e0.elapsed_time(e1) / iters
    f = unet_flops(width, n)
    out = {"width": width, "n": n, "params": int(net.n_params), "forward_ms": t_fwd,
           "train_step_ms": t_train, "forward_tflops": f / t_fwd / 1e9,
           "train_tflops": 3 * f / t_train / 1e9, "forward_gflop": f / 1e9,
           "mfma_peak_tflops": 2500.0, "forward_frac": f / t_fwd / 1e9 / 2500.0,
           "train_frac": 3 * f / t_train / 1e9 / 2500.0}
    log(f"[denoise] {json.dumps(out)}")
    return out


def main():
    import argparse
    import torch
    from . import engine as eng
    ap = argparse.ArgumentParser(description="train and evaluate the dose denoiser")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--test", type=int, default=20)
    ap.add_argument("--n-low", type=float, default=1e6)
    ap.add_argument("--n-high", type=float, default=1e9)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--out", default="out/denoise.json")
    ap.add_argument("--save", default="")
    ap.add_argument("--bench", action="store_true",
                    help="only time forward / training step at --width, --n")
    ap.add_argument("--iters", type=int, default=10, help="timed repetitions of --bench")
    args = ap.parse_args()
    if args.bench:
        print(json.dumps(bench_unet(args.width, args.n, args.iters)))
        return

    def log(m):
        print(m, file=sys.stderr, flush=True)

    model_src = wl.psr_model(20150306)
    t0 = time.perf_counter()
    train_pairs = make_pairs(range(1000, 1000 + args.train), int(args.n_low), int(args.n_high),
                             model_src, args.n, log)
    t_data = time.perf_counter() - t0
    log(f"[denoise] training data in {t_data:.1f} s")
    net = eng.UNet(args.width, args.n, args.n, args.n)
    from .unet_init import init_params
    net.set_params(init_params(7, args.width, net.n_params))
    t0 = time.perf_counter()
    hist = train(net, train_pairs, args.epochs, args.lr, log)
    t_train = time.perf_counter() - t0
    del train_pairs
    if args.save:
        np.save(args.save, net.get_params())
    # evaluation on held-out cases
    res = {"train_cases": args.train, "test_cases": args.test, "n_low": args.n_low,
           "n_high": args.n_high, "epochs": args.epochs, "loss_history": hist,
           "t_data_s": t_data, "t_train_s": t_train, "cases": []}
    vox = (0.25, 0.25, 0.25)
    for s in range(5000, 5000 + args.test):
        ph, beam = case_geometry(s, args.n)
        E = DoseEngine(model_src, ph, beam, s)
        t0 = time.perf_counter()
        ref, _ = E.dose(int(args.n_high), n_rep=1, seed_offset=9)
        torch.cuda.synchronize()
        t_ref = time.perf_counter() - t0
        rate = args.n_high / t_ref
        refn = ref.cpu().numpy()
        row = {"seed": s, "hist_per_s": rate}
        for nl in EVAL_COUNTS:
            d, sd = E.dose(int(nl), n_rep=4, seed_offset=int(nl) % 97 + 3)
            scale = float(d.max())
            inp = torch.stack([d / scale, torch.as_tensor(ph.density, device="cuda")]).contiguous()
            t0 = time.perf_counter()
            pred = net.forward(inp)
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - t0
            dn = (pred * scale).cpu().numpy()
            dp = d.cpu().numpy()
            row[f"{nl:.0e}"] = {
                "plain_rms": rms_percent(dp, refn), "denoised_rms": rms_percent(dn, refn),
                "plain_gamma": gamma_pass_rate(dp, refn, vox),
                "denoised_gamma": gamma_pass_rate(dn, refn, vox),
                "sigma_rel": sigma_rel(dp, sd.cpu().numpy()), "t_infer_s": t_inf}
        res["cases"].append(row)
        log(f"[denoise] test case {s}: " + json.dumps(row["1e+06"]))
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(res, f)
    print(json.dumps(summarize(res)))


def summarize(res):
    """Aggregate RMS / gamma and the time-to-1% comparison."""
    keys = tuple(f"{nl:.0e}" for nl in EVAL_COUNTS)
    out = {}
    for k in keys:
        rows = [c[k] for c in res["cases"]]
        out[k] = {m: float(np.mean([r[m] for r in rows]))
                  for m in ("plain_rms", "denoised_rms", "plain_gamma", "denoised_gamma",
                            "sigma_rel", "t_infer_s")}
    rate = float(np.mean([c["hist_per_s"] for c in res["cases"]]))
    # plain: histories to reach 1% mean sigma/D (sigma ~ 1/sqrt(N)), and the
    # RMS error (% of Dmax) a plain dose has at that count
    s1 = out["1e+06"]["sigma_rel"]
    n1 = 1e6 * (s1 / 0.01) ** 2
    rms_at_1pct = out["1e+06"]["plain_rms"] * math.sqrt(1e6 / n1)
    t_plain = n1 / rate
    # denoised: fewest histories whose denoised RMS reaches that error
    t_den = None
    n_den = None
    for k, nl in zip(keys, EVAL_COUNTS):
        if out[k]["denoised_rms"] <= rms_at_1pct:
            n_den = nl
            t_den = nl / rate + out[k]["t_infer_s"]
            break
    # equal error: the plain histories (RMS ~ 1/sqrt(N), fitted at 1e6) whose
    # RMS error equals each denoised dose's, and the time ratio
    equal = {}
    for k, nl in zip(keys, EVAL_COUNTS):
        n_eq = 1e6 * (out["1e+06"]["plain_rms"] / out[k]["denoised_rms"]) ** 2
        t_d = nl / rate + out[k]["t_infer_s"]
        equal[k] = {"denoised_rms": out[k]["denoised_rms"], "plain_histories_same_rms": n_eq,
                    "speedup": (n_eq / rate) / t_d}
    # stated RMS errors (% of Dmax): plain histories from the same fit, and
    # the fewest evaluated histories whose denoised dose reaches the error
    stated = {}
    for e in RMS_TARGETS:
        n_p = 1e6 * (out["1e+06"]["plain_rms"] / e) ** 2
        n_d = t_d = None
        for k, nl in zip(keys, EVAL_COUNTS):
            if out[k]["denoised_rms"] <= e:
                n_d, t_d = nl, nl / rate + out[k]["t_infer_s"]
                break
        stated[f"{e:g}"] = {"plain_histories": n_p, "plain_s": n_p / rate,
                            "denoised_histories": n_d, "denoised_s": t_d,
                            "speedup": (n_p / rate) / t_d if t_d else None}
    return {"per_history_count": out, "hist_per_s": rate,
            "time_to_1pct": {"rms_error_percent_of_dmax": rms_at_1pct,
                             "plain_histories": n1, "plain_s": t_plain,
                             "denoised_histories": n_den, "denoised_s": t_den},
            "time_to_rms": stated,
            "equal_rms": equal}


if __name__ == "__main__":
    main()
