"""Dose distributions of the 128^3 water workloads (5x5, 10x10 and 20x20 cm
fields at SSD 100): the central-axis depth dose and the crossline (x) and
inline (y) profiles at 1.5, 10 and 20 cm depth, each normalised to the
central-axis maximum, with field width (50 % level) and 80/20 penumbrae.

Usage: python -m paper_1503_01725_amd.report [--histories 1e8] [--out F]
Prints one JSON summary line; the full curves go to --out.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def _crossing(x, y, level, rising):
    """Linear-interpolated position where y crosses `level` (first rising /
    last falling crossing)."""
    idx = np.flatnonzero(y >= level)
    if idx.size == 0:
        return float("nan")
    i = idx[0] if rising else idx[-1]
    j = i - 1 if rising else i + 1
    if j < 0 or j >= len(y):
        return float(x[i])
    return float(x[j] + (level - y[j]) * (x[i] - x[j]) / (y[i] - y[j]))


def profile_metrics(x, p):
    """Field width at 50 % of the central value and mean 80/20 penumbra."""
    c = p[len(p) // 2 - 1:len(p) // 2 + 1].mean()
    q = p / c
    l50, r50 = _crossing(x, q, 0.5, True), _crossing(x, q, 0.5, False)
    l80, r80 = _crossing(x, q, 0.8, True), _crossing(x, q, 0.8, False)
    l20, r20 = _crossing(x, q, 0.2, True), _crossing(x, q, 0.2, False)
    return {"width50_cm": r50 - l50, "penumbra80_20_cm": 0.5 * ((l80 - l20) + (r20 - r80))}


def main():
    import torch
    from . import engine as eng
    from . import workloads as wl
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--histories", type=float, default=1e8)
    ap.add_argument("--replicas", type=int, default=10)
    ap.add_argument("--out", default="out/report_water128.json")
    args = ap.parse_args()
    full, summary = {}, {}
    for size in (5, 10, 20):
        W = wl.workload(f"water128_{size}")
        model = eng.Model(W.model)
        per = int(args.histories) // args.replicas
        plan = eng.Plan(model, W.beams, per, n_replica=args.replicas)
        ph = eng.Phantom(W.phantom)
        tally = eng.Tally(ph)
        prm = eng.transport_params()
        t0 = time.perf_counter()
        # the launch shape the autotuner picks for these fields on MI355X
        eng.run_plan(plan, ph, tally, prm, eng.run_opts(1 << 22, 24, seed=W.seed, lane_load=32,
                                                        sort_electrons=False, pipelines=2))
        d, s = tally.finalize(plan)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nx, ny, nz = W.phantom.shape_xyz
        vx, vy, vz = W.phantom.vox
        ox, oy, oz = W.phantom.origin
        D = d.cpu().numpy().reshape(nz, ny, nx)
        S = s.cpu().numpy().reshape(nz, ny, nx)
        cx, cy = nx // 2, ny // 2                   # x = 0 and y = 0 lie on a voxel face
        z = oz + (np.arange(nz) + 0.5) * vz
        x = ox + (np.arange(nx) + 0.5) * vx
        y = oy + (np.arange(ny) + 0.5) * vy
        cax = D[:, cy - 1:cy + 1, cx - 1:cx + 1].mean(axis=(1, 2))
        cax_s = np.sqrt((S[:, cy - 1:cy + 1, cx - 1:cx + 1] ** 2).sum(axis=(1, 2))) / 4
        dmax = float(cax.max())
        rec = {"z_cm": z.tolist(), "cax": (cax / dmax).tolist(),
               "cax_sigma_rel": (cax_s / np.maximum(cax, 1e-300)).tolist(), "profiles": {}}
        summ = {"seconds": dt, "histories_per_s": per * args.replicas / dt,
                "depth_of_max_cm": float(z[int(np.argmax(cax))]),
                "pdd10": float(np.interp(10.0, z, cax) / dmax),
                "pdd20": float(np.interp(20.0, z, cax) / dmax)}
        for depth in (1.5, 10.0, 20.0):
            k = int(np.clip(np.searchsorted(z, depth), 0, nz - 1))
            xp = D[k, cy - 1:cy + 1, :].mean(axis=0)
            yp = D[k, :, cx - 1:cx + 1].mean(axis=1)
            rec["profiles"][f"{depth:g}"] = {"x_cm": x.tolist(), "crossline": (xp / dmax).tolist(),
                                             "y_cm": y.tolist(), "inline": (yp / dmax).tolist()}
            summ[f"crossline_{depth:g}cm"] = profile_metrics(x, xp)
            summ[f"inline_{depth:g}cm"] = profile_metrics(y, yp)
        full[f"{size}x{size}"] = rec
        summary[f"{size}x{size}"] = summ
        print(f"[report] {size}x{size}: {json.dumps(summ)}", file=sys.stderr, flush=True)
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as f:
        json.dump({"summary": summary, "curves": full}, f)
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
