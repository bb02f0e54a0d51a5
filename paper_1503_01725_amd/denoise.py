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
# stated errors of the gated path (RMS over voxels above 10 % of Dmax, % of Dmax)
GATED_TARGETS = (4.0, 2.0, 1.0, 0.5)


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

    def dose(self, n_hist, n_rep=4, seed_offset=0, max_batch=1 << 20, fp64=False):
        """Dose and standard error (Gy per model particle, torch on the GPU;
        FP32 unless fp64)."""
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
        return (d, s) if fp64 else (d.float(), s.float())

    def dose_independent(self, n_hist, n_rep=4, seed_offset=0, max_batch=1 << 20):
        """Dose and standard error (FP64) from n_rep replicas whose plans hold
        N + 1, N + 2, ... histories (N = n_hist / n_rep).  The Eq. (3) counts
        of one plan are the same in each of its replicas, and with a few
        histories per phase-space-let their rounding leaves a fluence pattern
        that replicas of one plan share and their spread does not show;
        different N round differently, so the spread of these replicas covers
        it.  Normalised with the first plan's N (relative error < n_rep / N)."""
        import torch
        eng = self.eng
        per = max(1, n_hist // n_rep)
        tally = eng.Tally(self.phantom)
        plans = []
        for r in range(n_rep):
            plan = eng.Plan(self.model, [self.beam], per + 1 + r, n_replica=1)
            eng.run_plan(plan, self.phantom, tally, self.prm,
                         eng.run_opts(min(max_batch, max(4096, per)), 24, use_graph=False,
                                      seed=self.seed * 1000003 + seed_offset + 7919 * r))
            plans.append(plan)
        d, s = tally.finalize(plans[0])
        torch.cuda.synchronize()
        return d, s


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


GATE_CUTOFF = 0.1   # voxels judged: candidate dose above this fraction of its maximum
GATE_Z = 2.0        # standard errors on each side of the estimate for a decision
GATE_BLOCK = 4      # edge of the voxel blocks of the correlation-robust standard error


def gate_stats(cand, plain, plain_sigma, cutoff=GATE_CUTOFF, z=GATE_Z, block=GATE_BLOCK):
    """The plain engine's judgement of a candidate dose (psl_dose_gate).

    M is the candidate's largest mean over block^3-voxel blocks.  mse: mean
    of (cand - plain)^2 - sigma^2 over the voxels where the candidate exceeds
    `cutoff` of M, an unbiased estimate of the candidate's mean squared error
    against the true dose; se: its standard error from the blocks (noise
    correlated within a block counted); dmax: the plain dose's mean over the
    candidate's top region (blocks whose candidate mean is >= 95 % of M), an
    unbiased reading of the true dose there that a spurious hot spot of the
    candidate lowers rather than raises.  Returned in % of dmax:
    the estimate, its band estimate_lo / estimate_hi at z standard errors, and
    the plain dose's own RMS standard error over the same voxels."""
    import ctypes as C
    import torch
    from . import _native as N
    shape = tuple(plain.shape) if plain.dim() == 3 else (1, 1, plain.numel())
    assert cand.numel() == plain.numel() == plain_sigma.numel()
    assert cand.dtype == torch.float32 and plain.dtype == plain_sigma.dtype == torch.float64
    cand, plain, plain_sigma = cand.contiguous(), plain.contiguous(), plain_sigma.contiguous()
    out = np.zeros(10)
    nz, ny, nx = shape
    N.check(N.lib().psl_dose_gate(cand.data_ptr(), plain.data_ptr(), plain_sigma.data_ptr(),
                                  nx, ny, nz, block, cutoff, out.ctypes.data_as(N.dp),
                                  C.c_void_p(int(torch.cuda.current_stream().cuda_stream))))
    n_c, cmax, sd2, ss2, st2, stn, sn2, n_top, sum_top, n_blk = out
    dmax = sum_top / n_top if n_top > 0 else 0.0
    if n_c == 0 or not dmax > 0:
        inf = float("inf")
        return {"voxels": int(n_c), "estimate": inf, "estimate_lo": inf, "estimate_hi": inf,
                "plain_rms": inf, "mse": inf, "se": inf, "dmax": dmax}
    mse = (sd2 - ss2) / n_c
    var = (st2 - 2.0 * mse * stn + mse * mse * sn2) / (n_c * n_c)
    if n_blk > 1:
        var *= n_blk / (n_blk - 1.0)
    se = float(np.sqrt(max(var, 0.0)))
    pct = 100.0 / dmax
    root = lambda v: pct * float(np.sqrt(max(v, 0.0)))
    return {"voxels": int(n_c), "blocks": int(n_blk), "dmax": float(dmax),
            "candidate_max": float(cmax), "mse": float(mse), "se": se,
            "estimate": root(mse), "estimate_lo": root(mse - z * se),
            "estimate_hi": root(mse + z * se), "plain_rms": root(ss2 / n_c)}


def gated_dose(net, E, density, n_input, target_rms, n_judge=None, judge_reps=4,
               seed_offsets=(11, 12, 13), max_rounds=3):
    """The denoised dose with the plain engine as its judge and fallback.

    1. A plain dose of n_input histories (one replica) is the network's input.
    2. An independent plain dose (judge_reps replicas of distinct history
       counts, DoseEngine.dose_independent, other random numbers; n_judge
       histories, default 4 n_input) and its standard error judge the
       prediction (gate_stats): the mean of (denoised - judge)^2 - sigma^2
       estimates the denoised dose's squared error against the true dose.
    3. If the estimate plus two standard errors is within target_rms (% of
       Dmax) the denoised dose is returned.  If the estimate minus two
       standard errors exceeds it, or the judge would have to grow to half
       the plain run the target needs, the plain engine takes over.
       Otherwise (the judge too noisy to decide) the judge runs again with
       4x the histories, at most max_rounds times.
    4. The fallback: the plain engine runs to target_rms, with its histories
       scaled from the judge's own RMS error (sigma ~ N^-1/2) and extended
       until the run's own RMS standard error meets target_rms; the plain
       dose is returned.
    Returns (dose on the device, FP32 or FP64; info dict with the branch
    taken, the histories run and the gate figures)."""
    import torch
    n_judge = int(n_judge or 4 * n_input)
    t0 = time.perf_counter()
    d_in, _ = E.dose(int(n_input), n_rep=1, seed_offset=seed_offsets[0])
    scale = float(d_in.max())
    if not scale > 0:
        raise ValueError("the plain input dose is zero everywhere")
    dens = torch.as_tensor(density, dtype=torch.float32, device="cuda")
    inp = torch.stack([d_in / scale, dens]).contiguous()
    pred = net.forward(inp) * scale
    spent = int(n_input)
    rounds = []
    for rnd in range(max_rounds):
        judge, jsig = E.dose_independent(n_judge, n_rep=judge_reps,
                                         seed_offset=seed_offsets[1] + 997 * rnd)
        spent += n_judge
        g = gate_stats(pred, judge, jsig)
        rounds.append({"n_judge": n_judge, "estimate": g["estimate"],
                       "estimate_lo": g["estimate_lo"], "estimate_hi": g["estimate_hi"],
                       "plain_rms": g["plain_rms"]})
        if g["estimate_hi"] <= target_rms:
            torch.cuda.synchronize()
            return pred, {"gate": g, "rounds": rounds, "target_rms": float(target_rms),
                          "n_input": int(n_input), "branch": "denoised", "histories": spent,
                          "seconds": time.perf_counter() - t0, "candidate": pred}
        n_plain_need = n_judge * (g["plain_rms"] / target_rms) ** 2
        if g["estimate_lo"] > target_rms or 4 * n_judge > 0.5 * n_plain_need:
            break
        n_judge *= 4
    info = {"gate": g, "rounds": rounds, "target_rms": float(target_rms),
            "n_input": int(n_input), "candidate": pred}
    # the plain engine to the stated error: histories scaled from the judge's
    # own error, then from the run's own (its high-dose region) until that
    # meets the target
    n_plain = max(int(np.ceil(n_judge * (g["plain_rms"] / target_rms) ** 2)), judge_reps)
    for attempt in range(4):
        d, s = E.dose_independent(n_plain, n_rep=judge_reps,
                                  seed_offset=seed_offsets[2] + 101 * attempt)
        spent += n_plain
        own = gate_stats(d.float(), d, s)["plain_rms"]
        if own <= target_rms:
            break
        n_plain = int(np.ceil(n_plain * 1.1 * (own / target_rms) ** 2))
    torch.cuda.synchronize()
    info.update(branch="plain", n_plain=n_plain, plain_rms=own, histories=spent,
                seconds=time.perf_counter() - t0, sigma=s)
    return d, info


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


def measure_time_to_1pct(k, n=128, n_high=1e9, n0=1e6, log=None):
    """The plain engine's time to 1 % sigma, run rather than extrapolated, on
    the first k test cases: sigma_rel at n0 histories predicts
    N = n0 (sigma_rel / 0.01)^2; the engine then runs N histories (4
    replicas, timed after a warm-up run of the same plan) and sigma_rel is
    measured on that dose; while it is still above 1 %, N grows by the same
    rule with a 2 % margin (at most two more runs).  Also the RMS error (% of
    Dmax, all voxels) of that dose against an n_high reference."""
    import torch
    log = log or (lambda m: print(m, file=sys.stderr, flush=True))
    from . import engine as eng
    model_src = wl.psr_model(20150306)
    rows = []
    for s in range(5000, 5000 + k):
        ph, beam = case_geometry(s, n)
        E = DoseEngine(model_src, ph, beam, s)
        d0, s0 = E.dose(int(n0), n_rep=4, seed_offset=3)
        n_pred = n0 * (sigma_rel(d0.cpu().numpy(), s0.cpu().numpy()) / 0.01) ** 2
        runs = []
        n_run = int(math.ceil(n_pred))
        for _ in range(3):
            per = max(1, n_run // 4)
            plan = eng.Plan(E.model, [beam], per, n_replica=4)
            tally = eng.Tally(E.phantom)
            opts = eng.run_opts(1 << 22, 24, use_graph=False, seed=s * 1000003 + 17,
                                lane_load=32, pipelines=2, sort_electrons=False)
            eng.run_plan(plan, E.phantom, tally, E.prm, opts)      # warm-up
            torch.cuda.synchronize()
            tally.op(eng.N.PSL_TALLY_RESET)
            t0 = time.perf_counter()
            eng.run_plan(plan, E.phantom, tally, E.prm, opts)
            d, sd = tally.finalize(plan)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            dn, sdn = d.float().cpu().numpy(), sd.float().cpu().numpy()
            sr = sigma_rel(dn, sdn)
            runs.append({"histories": per * 4, "sigma_rel": sr, "seconds": t})
            if sr <= 0.01:
                break
            n_run = int(math.ceil(per * 4 * (sr / 0.01) ** 2 * 1.02))
        ref = E.dose(int(n_high), n_rep=1, seed_offset=9)[0].cpu().numpy()
        row = {"seed": s, "predicted_histories": n_pred, "runs": runs,
               "rms_percent_dmax": rms_percent(dn, ref),
               "met": runs[-1]["sigma_rel"] <= 0.01}
        rows.append(row)
        log(f"[time-to-1%] case {s}: " + json.dumps(row))
    last = [r["runs"][-1] for r in rows]
    return {"cases": rows,
            "mean_histories": float(np.mean([r["histories"] for r in last])),
            "mean_seconds": float(np.mean([r["seconds"] for r in last])),
            "mean_sigma_rel": float(np.mean([r["sigma_rel"] for r in last])),
            "mean_rms_percent_dmax": float(np.mean([r["rms_percent_dmax"] for r in rows])),
            "met": int(sum(r["met"] for r in rows)),
            "mean_predicted_histories": float(np.mean([r["predicted_histories"] for r in rows]))}


def rms_percent_region(d, ref, cutoff=GATE_CUTOFF):
    """Eq. (10) over the voxels where the reference exceeds `cutoff` of its
    maximum, in % of that maximum (the region and scale the gate judges)."""
    m = ref > cutoff * ref.max()
    return 100.0 * float(np.sqrt(np.mean((d[m] - ref[m]).astype(np.float64) ** 2))) / float(ref.max())


def main():
    import argparse
    import torch
    from . import engine as eng
    ap = argparse.ArgumentParser(description="train and evaluate the dose denoiser")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--val", type=int, default=5,
                    help="validation cases that choose the gated input size per stated error")
    ap.add_argument("--test", type=int, default=20)
    ap.add_argument("--n-low", type=float, default=1e6)
    ap.add_argument("--n-high", type=float, default=1e9)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-decay", type=float, default=0.5,
                    help="learning rate at the last epoch as a fraction of --lr (geometric)")
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--out", default="out/denoise.json")
    ap.add_argument("--save", default="")
    ap.add_argument("--bench", action="store_true",
                    help="only time forward / training step at --width, --n")
    ap.add_argument("--iters", type=int, default=10, help="timed repetitions of --bench")
    ap.add_argument("--time-to-1pct", type=int, default=0, metavar="K",
                    help="only measure the plain engine's time to 1 %% sigma on K test cases")
    args = ap.parse_args()
    if args.bench:
        print(json.dumps(bench_unet(args.width, args.n, args.iters)))
        return
    if args.time_to_1pct:
        print(json.dumps(measure_time_to_1pct(args.time_to_1pct, args.n, args.n_high)))
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
    hist = train(net, train_pairs, args.epochs, args.lr, log, lr_decay=args.lr_decay)
    t_train = time.perf_counter() - t0
    del train_pairs
    if args.save:
        np.save(args.save, net.get_params())
    res = {"train_cases": args.train, "val_cases": args.val, "test_cases": args.test,
           "n_low": args.n_low, "n_high": args.n_high, "epochs": args.epochs,
           "loss_history": hist, "t_data_s": t_data, "t_train_s": t_train, "cases": []}
    vox = (0.25, 0.25, 0.25)
    dens_of = lambda ph: torch.as_tensor(ph.density, device="cuda")

    def denoise_once(E, ph, nl, seed_offset):
        d, _ = E.dose(int(nl), n_rep=1, seed_offset=seed_offset)
        scale = float(d.max())
        inp = torch.stack([d / scale, dens_of(ph)]).contiguous()
        return (net.forward(inp) * scale)

    # validation (seeds of their own): the denoised error per input size
    val = {f"{nl:.0e}": [] for nl in EVAL_COUNTS}
    for s in range(7000, 7000 + args.val):
        ph, beam = case_geometry(s, args.n)
        E = DoseEngine(model_src, ph, beam, s)
        ref = E.dose(int(args.n_high), n_rep=1, seed_offset=9)[0].cpu().numpy()
        for nl in EVAL_COUNTS:
            dn_ = denoise_once(E, ph, nl, 7).cpu().numpy()
            val[f"{nl:.0e}"].append(rms_percent_region(dn_, ref))
        log(f"[denoise] validation case {s}")
    val_mean = {k: float(np.mean(v)) for k, v in val.items()}
    # input size of the gated path per stated error: the fewest histories
    # whose validation denoised error is at most 0.8 of it (None: the
    # denoiser does not reach it, the gate will hand over to the plain engine)
    policy = {}
    for e in GATED_TARGETS:
        policy[f"{e:g}"] = next((nl for nl in EVAL_COUNTS if val_mean[f"{nl:.0e}"] <= 0.8 * e),
                                None)
    res["validation_denoised_rms_region"] = val_mean
    res["gated_input_policy"] = policy
    log(f"[denoise] validation {json.dumps(val_mean)} policy {json.dumps(policy)}")
    for s in range(5000, 5000 + args.test):
        ph, beam = case_geometry(s, args.n)
        E = DoseEngine(model_src, ph, beam, s)
        t0 = time.perf_counter()
        ref, _ = E.dose(int(args.n_high), n_rep=1, seed_offset=9)
        torch.cuda.synchronize()
        t_ref = time.perf_counter() - t0
        rate = args.n_high / t_ref
        refn = ref.cpu().numpy()
        row = {"seed": s, "hist_per_s": rate, "gated": {}}
        for nl in EVAL_COUNTS:
            d, sd = E.dose(int(nl), n_rep=4, seed_offset=int(nl) % 97 + 3)
            scale = float(d.max())
            inp = torch.stack([d / scale, dens_of(ph)]).contiguous()
            t0 = time.perf_counter()
            pred = net.forward(inp)
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - t0
            dn_ = (pred * scale).cpu().numpy()
            dp = d.cpu().numpy()
            row[f"{nl:.0e}"] = {
                "plain_rms": rms_percent(dp, refn), "denoised_rms": rms_percent(dn_, refn),
                "plain_rms_region": rms_percent_region(dp, refn),
                "denoised_rms_region": rms_percent_region(dn_, refn),
                "plain_gamma": gamma_pass_rate(dp, refn, vox),
                "denoised_gamma": gamma_pass_rate(dn_, refn, vox),
                "sigma_rel": sigma_rel(dp, sd.cpu().numpy()), "t_infer_s": t_inf}
        # the gated path at each stated error (region RMS, % of Dmax)
        for e in GATED_TARGETS:
            n_in = policy[f"{e:g}"]
            if n_in is None:
                # the denoiser does not reach e on validation: plain engine,
                # histories from the plain error at 1e6 (sigma ~ N^-1/2)
                n_p = int(np.ceil(1e6 * (row["1e+06"]["plain_rms_region"] / e) ** 2))
                t0 = time.perf_counter()
                dd, _ = E.dose(n_p, n_rep=4, seed_offset=41)
                torch.cuda.synchronize()
                info = {"branch": "plain (policy)", "histories": n_p,
                        "seconds": time.perf_counter() - t0}
            else:
                dd, info = gated_dose(net, E, ph.density, n_in, e)
            got = rms_percent_region(dd.float().cpu().numpy(), refn)
            row["gated"][f"{e:g}"] = {"branch": info["branch"], "histories": info["histories"],
                                      "seconds": info["seconds"], "rms_region": got,
                                      "met": got <= e,
                                      "estimate": info.get("gate", {}).get("estimate")}
        res["cases"].append(row)
        log(f"[denoise] test case {s}: " + json.dumps(row["1e+06"]) + " gated " +
            json.dumps(row["gated"]))
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
    # the gated path: per stated error, the branch taken, the fraction of
    # cases whose returned dose meets it, histories and time, against the
    # plain engine's histories to the same error (fit at 1e6 per case)
    gated = {}
    if res["cases"] and "gated" in res["cases"][0]:
        n_high = float(res.get("n_high", 1e9))
        t_inf = out["1e+06"]["t_infer_s"]
        for e in GATED_TARGETS:
            key = f"{e:g}"
            rows = [c["gated"][key] for c in res["cases"]]
            n_plain = [1e6 * (c["1e+06"]["plain_rms_region"] / e) ** 2 for c in res["cases"]]
            # the reference's own noise, from the same N^-1/2 fit, taken out of
            # the returned dose's error before comparing it with the stated one
            ref_noise = [c["1e+06"]["plain_rms_region"] * math.sqrt(1e6 / n_high)
                         for c in res["cases"]]
            err = [math.sqrt(max(r["rms_region"] ** 2 - q ** 2, 0.0))
                   for r, q in zip(rows, ref_noise)]
            h_g = float(np.mean([r["histories"] for r in rows]))
            den = [r["branch"] == "denoised" for r in rows]
            # modelled time: histories at the measured rate plus the inference
            # of the cases that ran the network
            t_model = h_g / rate + t_inf * float(np.mean([r["branch"] != "plain (policy)"
                                                          for r in rows]))
            gated[key] = {"denoised_fraction": float(np.mean(den)),
                          "met_fraction": float(np.mean([x <= e for x in err])),
                          "mean_rms_region": float(np.mean([r["rms_region"] for r in rows])),
                          "mean_error_region": float(np.mean(err)),
                          "reference_noise_region": float(np.mean(ref_noise)),
                          "histories": h_g, "seconds_measured": float(np.mean(
                              [r["seconds"] for r in rows])),
                          "seconds_model": t_model,
                          "plain_histories": float(np.mean(n_plain)),
                          "plain_s": float(np.mean(n_plain)) / rate,
                          "speedup_histories": float(np.mean(n_plain)) / h_g,
                          "speedup_time_model": float(np.mean(n_plain)) / rate / t_model}
    for k in keys:
        if "plain_rms_region" in res["cases"][0][k]:
            for m in ("plain_rms_region", "denoised_rms_region"):
                out[k][m] = float(np.mean([c[k][m] for c in res["cases"]]))
    return {"per_history_count": out, "hist_per_s": rate, "gated": gated,
            "gated_input_policy": res.get("gated_input_policy"),
            "time_to_1pct": {"rms_error_percent_of_dmax": rms_at_1pct,
                             "plain_histories": n1, "plain_s": t_plain,
                             "denoised_histories": n_den, "denoised_s": t_den},
            "time_to_rms": stated,
            "equal_rms": equal}


if __name__ == "__main__":
    main()
