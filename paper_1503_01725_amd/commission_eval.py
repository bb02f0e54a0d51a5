"""Commissioning in the shape of the paper's experiment (Sec. 2.2, Sec. 3.2;
Tables 2-3, Fig. 7), against a synthetic measured beam.

* Model: the synthetic PSR model with 10 energy bins and widened to cover a
  40 x 40 cm field at the plane (30 rings of 1 cm, PSL grid 60 cm).
* Bases (Sec. 2.2.3): one correction factor per photon PSR (primary and
  scatter, every energy bin and ring) and one per electron energy bin (the
  electron PSRs of a bin form one effective unit).
* Commissioning data (Sec. 3.2): central-axis depth dose and inline and
  crossline profiles at 1.5, 10 and 20 cm of a 40 x 40 and a 5 x 5 cm field
  at SSD 100 in a 64 cm water cube (0.5 cm voxels).
* Measured beam: the same model with its PSR weights perturbed smoothly
  (primary horn and energy tilt, scatter level, electron spectrum and a
  radial electron tilt that the per-bin electron units cannot represent),
  simulated independently: it stands in for the linac measurements, with
  model error and Monte Carlo noise of its own.
* Fit: Eq. (8), x >= 0 by commission_nnls, no regularisation.
* Evaluation on 40, 20, 10, 5 and 2 cm fields: the commissioned model and the
  uncommissioned one against the measured beam, with the paper's metrics
  (Eq. 9): RMS and maximum difference in % of the measured maximum in the
  low-gradient regions (depth dose past the build-up, inner and outer
  profile regions), distance to agreement in the high-gradient regions
  (build-up, penumbra), and output factors.  Each model is calibrated to the
  measured dose at 10 cm depth on the axis of the 10 x 10 field.

Usage: python -m paper_1503_01725_amd.commission_eval [--hist-per-basis 1e7]
       [--hist-per-field 3e9] [--hist-measured 1e10]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time

import numpy as np

FIELDS_COMMISSION = (40.0, 5.0)
FIELDS_EVAL = (40.0, 20.0, 10.0, 5.0, 2.0)
DEPTHS = (1.5, 10.0, 20.0)
N_VOX, VOX = 128, 0.5


# --------------------------------------------------------------------------
# Model, measured beam, bases
# --------------------------------------------------------------------------
def wide_model(seed: int):
    """10 energy bins (the paper's bins are a tenth of the maximum energy),
    30 rings of 1 cm and a 60 cm PSL grid of 0.5 cm: 610 bases, fewer than
    the 1792 commissioning rows, so that Eq. (8) is overdetermined."""
    from . import workloads as wl
    return wl.psr_model(seed, n_ebin=10, n_ring=30, ring_dr=1.0, n_psl=120, psl_dx=0.5)


def measured_model(model, strength: float = 1.0):
    """The measured beam: smooth perturbations of the PSR weights (s, b, j)."""
    e_mid = model.e_lo + (np.arange(model.n_ebin) + 0.5) * model.e_width
    r_mid = (np.arange(model.n_ring) + 0.5) * model.ring_dr
    et = (e_mid - e_mid.mean()) / (e_mid.max() - e_mid.min())     # -0.5 .. 0.5
    rt = r_mid / r_mid.max()                                      # 0 .. 1
    p = np.ones_like(model.w_psr)
    p[0] = (1.0 + 0.20 * strength * et)[:, None] * (1.0 + 0.12 * strength * rt ** 2)[None, :]
    p[1] = (1.0 + 0.30 * strength) * (1.0 - 0.15 * strength * rt)[None, :]
    p[2] = (1.0 - 0.60 * strength * et)[:, None] * (1.0 + 0.30 * strength * rt)[None, :]
    return dataclasses.replace(model, w_psr=np.ascontiguousarray(model.w_psr * p))


def basis_map(model) -> np.ndarray:
    """Basis id per PSR: photon PSRs one each, electron PSRs one per energy bin."""
    nb, nr = model.n_ebin, model.n_ring
    m = np.empty((3, nb, nr), dtype=np.int64)
    for s in (0, 1):
        m[s] = s * nb * nr + np.arange(nb)[:, None] * nr + np.arange(nr)[None, :]
    m[2] = 2 * nb * nr + np.arange(nb)[:, None]
    return np.ascontiguousarray(m, dtype=np.uint16)


def n_basis(model) -> int:
    return 2 * model.n_ebin * model.n_ring + model.n_ebin


def smoothness_rows(model) -> np.ndarray:
    """First differences of the correction factors between neighbouring rings
    (same photon sub-source and energy bin): one row (+1, -1) per pair."""
    bm = basis_map(model).astype(np.int64)
    pairs = [(bm[s, b, r], bm[s, b, r + 1]) for s in (0, 1) for b in range(model.n_ebin)
             for r in range(model.n_ring - 1)]
    D = np.zeros((len(pairs), n_basis(model)))
    for k, (i, j) in enumerate(pairs):
        D[k, i], D[k, j] = 1.0, -1.0
    return D


def corrected_model(model, x_basis: np.ndarray):
    """The model with each PSR weight times its basis' correction factor."""
    f = x_basis[basis_map(model).astype(np.int64)]
    return dataclasses.replace(model, w_psr=np.ascontiguousarray(model.w_psr * f))


# --------------------------------------------------------------------------
# Curves (depth dose and profiles) on the water cube
# --------------------------------------------------------------------------
def curve_voxels(n: int = N_VOX, vox: float = VOX):
    """(name, [(iz, iy, ix)...], positions in cm): the axis depth dose and the
    inline (y) and crossline (x) profiles at DEPTHS."""
    c = n // 2
    pos = (np.arange(n) + 0.5) * vox - n * vox / 2.0
    depth = (np.arange(n) + 0.5) * vox
    out = [("pdd", [(k, c, c) for k in range(n)], depth)]
    for d in DEPTHS:
        k = int(math.floor(d / vox))
        out.append((f"inline_{d:g}", [(k, j, c) for j in range(n)], pos))
        out.append((f"crossline_{d:g}", [(k, c, i) for i in range(n)], pos))
    return out


def index_map(n: int = N_VOX, vox: float = VOX):
    """Voxel -> row + 1 over the curves' voxels (raster order) and, per
    curve, its row indices."""
    sel = np.zeros((n, n, n), dtype=bool)
    for _, vs, _ in curve_voxels(n, vox):
        for v in vs:
            sel[v] = True
    imap = np.zeros((n, n, n), dtype=np.int32)
    idx = np.flatnonzero(sel.ravel())
    imap.ravel()[idx] = np.arange(1, idx.size + 1, dtype=np.int32)
    rows = {name: np.array([imap[v] - 1 for v in vs]) for name, vs, _ in curve_voxels(n, vox)}
    return imap, int(idx.size), rows


def curves_of_grid(dose: np.ndarray, n: int = N_VOX, vox: float = VOX) -> dict:
    return {name: np.array([dose[v] for v in vs]) for name, vs, _ in curve_voxels(n, vox)}


def positions(n: int = N_VOX, vox: float = VOX) -> dict:
    return {name: p for name, _, p in curve_voxels(n, vox)}


# --------------------------------------------------------------------------
# Metrics (Eq. 9 and the distance to agreement)
# --------------------------------------------------------------------------
def dta(pos: np.ndarray, meas: np.ndarray, calc: np.ndarray, sel: np.ndarray,
        window: float = 2.0) -> np.ndarray:
    """For each selected measured point x: the smallest |x - y| <= window with
    calc(y) = meas(x), calc linearly interpolated between the points and
    extended linearly past the first and last (the surface lies half a voxel
    before the first depth); `window` where there is none."""
    out = np.full(int(sel.sum()), float(window))
    h0, h1 = pos[1] - pos[0], pos[-1] - pos[-2]
    xp = np.concatenate([[pos[0] - h0], pos, [pos[-1] + h1]])
    cp = np.concatenate([[2 * calc[0] - calc[1]], calc, [2 * calc[-1] - calc[-2]]])
    for k, i in enumerate(np.flatnonzero(sel)):
        f = cp - meas[i]
        cand = list(np.abs(xp[f == 0] - pos[i]))
        s = np.flatnonzero(np.sign(f[:-1]) * np.sign(f[1:]) < 0)
        if s.size:
            y = xp[s] + (xp[s + 1] - xp[s]) * f[s] / (f[s] - f[s + 1])
            cand.extend(np.abs(y - pos[i]))
        if cand:
            out[k] = min(float(window), min(cand))
    return out


def _rms_max(meas, calc, sel, norm):
    d = (calc[sel] - meas[sel]) / norm * 100.0
    if d.size == 0:
        return None, None
    return float(np.sqrt(np.mean(d ** 2))), float(np.abs(d).max())


def depth_dose_metrics(depth, meas, calc) -> dict:
    """Build-up (depths before the measured maximum): DTA; past it: RMS and
    maximum difference in % of the measured maximum."""
    kmax = int(np.argmax(meas))
    dmax = float(meas[kmax])
    build = np.arange(depth.size) < kmax
    after = (np.arange(depth.size) >= kmax) & (meas > 0.0)
    after[-2:] = False                 # the phantom's exit face
    t = dta(depth, meas, calc, build) if build.any() else np.array([0.0])
    rms, mx = _rms_max(meas, calc, after, dmax)
    return {"dta_mean_cm": float(np.mean(t)), "dta_max_cm": float(np.max(t)),
            "rms_pct": rms, "max_pct": mx}


def profile_metrics(pos, meas, calc) -> dict:
    """Regions by the measured profile relative to its axis value: inner
    (>= 80 %), penumbra (20-80 %, DTA) and outer (< 20 %, away from the
    phantom's side faces)."""
    c = int(np.argmin(np.abs(pos)))
    ref = float(meas[c])
    r = meas / ref
    inner = r >= 0.8
    pen = (r >= 0.2) & (r < 0.8)
    outer = r < 0.2
    outer[:2] = outer[-2:] = False
    ri, mi = _rms_max(meas, calc, inner, ref)
    ro, mo = _rms_max(meas, calc, outer, ref)
    t = dta(pos, meas, calc, pen) if pen.any() else np.array([0.0])
    return {"inner_rms_pct": ri, "inner_max_pct": mi, "outer_rms_pct": ro, "outer_max_pct": mo,
            "penumbra_dta_mean_cm": float(np.mean(t)), "penumbra_dta_max_cm": float(np.max(t))}


def field_metrics(pos: dict, meas: dict, calc: dict) -> dict:
    out = {"pdd": depth_dose_metrics(pos["pdd"], meas["pdd"], calc["pdd"])}
    for name in meas:
        if name != "pdd":
            out[name] = profile_metrics(pos[name], meas[name], calc[name])
    return out


def output_factor(curves: dict, ref_curves: dict) -> float:
    """Axis dose at 10 cm depth relative to that of the 10 x 10 field."""
    k = int(math.floor(10.0 / VOX))
    return float(curves["pdd"][k] / ref_curves["pdd"][k])


# --------------------------------------------------------------------------
# GPU runs
# --------------------------------------------------------------------------
def field_dose(eng, model_src, size, n_hist, seed, phantom, opts, prm, replicas=4):
    """Dose grid (Gy per model particle) of one square field at SSD 100."""
    from . import workloads as wl
    model = eng.Model(model_src)
    plan = eng.Plan(model, [wl.square_beam(size)], int(n_hist) // replicas, n_replica=replicas)
    tally = eng.Tally(phantom)
    eng.run_plan(plan, phantom, tally, prm, opts)
    dose, sig = tally.finalize(plan)
    return dose.cpu().numpy(), sig.cpu().numpy()


def basis_doses(eng, model_src, fields, hist_per_basis, seed, phantom, opts, prm):
    """A: rows x (field, basis) doses through the index-map tally, one run."""
    from . import workloads as wl
    imap, n_rows, rows = index_map()
    nb = n_basis(model_src)
    model = eng.Model(model_src)
    plan = eng.Plan(model, [wl.square_beam(s) for s in fields], 0, n_replica=1,
                    basis_map=basis_map(model_src), hist_per_basis=int(hist_per_basis))
    tally = eng.Tally(phantom, index_map=imap, n_rows=n_rows, n_cols=len(fields) * nb)
    t0 = time.perf_counter()
    eng.run_plan(plan, phantom, tally, prm, opts)
    A_dev, _ = tally.finalize(plan)
    A = A_dev.cpu().numpy().reshape(n_rows, len(fields) * nb)
    return A, rows, plan.n_hist, time.perf_counter() - t0


def scaled_system(A: np.ndarray, b: np.ndarray, D=None, smooth: float = 0.0,
                  min_sens: float = 0.0):
    """The least-squares system the solver sees: the used columns scaled to
    unit norm, then the whole system divided by b's maximum, so y = x * cn
    over the used bases.  A column is used if some row sees it and, with
    min_sens > 0, if its norm is at least min_sens times the median norm of
    the seen columns (the data barely constrain the others); an unused basis
    keeps its factor 1, and its dose moves to the right-hand side.  With
    smooth > 0 the rows sqrt(smooth) * D follow.  Then
    |A1 y - b1|^2 = |A x - b|^2 / scale^2 + smooth |D x|^2."""
    norms = np.linalg.norm(A, axis=0)
    used = norms > 0
    if min_sens > 0.0:
        used = norms > min_sens * float(np.median(norms[used]))
    Au = A[:, used]
    cn = norms[used]
    scale = float(np.abs(b).max())
    A1, b1 = Au / cn / scale, (b - A[:, ~used].sum(axis=1)) / scale
    if D is not None and smooth > 0.0:
        keep = np.abs(D[:, used]).sum(axis=1) > 0
        w = np.sqrt(smooth)
        A1 = np.vstack([A1, w * (D[:, used] / cn)[keep]])
        b1 = np.concatenate([b1, -w * D[:, ~used].sum(axis=1)[keep]])
    return A1, b1, used, cn, scale


def fit(eng, A: np.ndarray, b: np.ndarray, max_iter: int, D=None, smooth: float = 0.0,
        min_sens: float = 0.0):
    """Eq. (8) on the scaled system (plus the smoothness rows when smooth > 0);
    bases left out of it keep their factor 1."""
    A1, b1, used, cn, _ = scaled_system(A, b, D, smooth, min_sens)
    y, rep = eng.commission_nnls(A1, b1, x0=np.ones(int(used.sum())) * cn, max_iter=max_iter)
    x = np.ones(A.shape[1])
    x[used] = y / cn
    return x, used, rep


def evaluate(hist_per_basis=1e7, hist_per_field=3e9, hist_measured=1e10, max_iter=300000,
             seed=20150306, smooth=0.0, log=print, min_sens=0.0) -> dict:
    """The whole experiment; returns the result dictionary printed by main()."""
    from . import engine as eng
    from . import workloads as wl
    t_start = time.perf_counter()
    src = wide_model(seed)
    meas_src = measured_model(src)
    phantom = eng.Phantom(wl.water_phantom(N_VOX, VOX))
    prm = eng.transport_params()
    opts = eng.run_opts(1 << 22, 24, use_graph=True, sort_electrons=False, seed=seed,
                        lane_load=32, pipelines=2)
    pos = positions()

    # 1. basis doses of the commissioning fields (the model as built)
    A, rows, n_a, t_a = basis_doses(eng, src, FIELDS_COMMISSION, hist_per_basis, seed, phantom,
                                    opts, prm)
    log(f"[commission_eval] basis doses: {n_a} histories in {t_a:.2f} s")
    # 2. the measured beam on every field, the uncommissioned model on every field
    meas, ref = {}, {}
    for s in FIELDS_EVAL:
        d, _ = field_dose(eng, meas_src, s, hist_measured, seed + 1, phantom, opts, prm)
        meas[s] = curves_of_grid(d)
        d, _ = field_dose(eng, src, s, hist_per_field, seed + 2, phantom, opts, prm)
        ref[s] = curves_of_grid(d)
        log(f"[commission_eval] field {s:g}: measured and reference doses")
    # 3. Eq. (8): stacked rows of both commissioning fields
    nb = n_basis(src)
    names = list(rows)
    blocks, bvec = [], []
    for f, s in enumerate(FIELDS_COMMISSION):
        for name in names:
            blocks.append(A[rows[name], f * nb:(f + 1) * nb])
            bvec.append(meas[s][name])
    As, bs = np.vstack(blocks), np.concatenate(bvec)
    t0 = time.perf_counter()
    x, used, rep = fit(eng, As, bs, max_iter, smoothness_rows(src), smooth, min_sens)
    t_fit = time.perf_counter() - t0
    log(f"[commission_eval] NNLS: {rep['iters']} iterations, {t_fit:.2f} s")
    # 4. the commissioned model on every field
    com_src = corrected_model(src, x)
    com = {}
    for s in FIELDS_EVAL:
        d, _ = field_dose(eng, com_src, s, hist_per_field, seed + 3, phantom, opts, prm)
        com[s] = curves_of_grid(d)
    # 5. calibration at 10 cm on the 10 x 10 axis, metrics, output factors
    k10 = int(math.floor(10.0 / VOX))

    def calibrated(cur):
        c = meas[10.0]["pdd"][k10] / cur[10.0]["pdd"][k10]
        return {s: {n: v * c for n, v in cur[s].items()} for s in cur}

    ref_c, com_c = calibrated(ref), calibrated(com)
    result = {"fields": {}, "output_factor_diff_pct": {"reference": {}, "commissioned": {}}}
    for s in FIELDS_EVAL:
        result["fields"][f"{s:g}x{s:g}"] = {"reference": field_metrics(pos, meas[s], ref_c[s]),
                                            "commissioned": field_metrics(pos, meas[s], com_c[s])}
        of_m = output_factor(meas[s], meas[10.0])
        result["output_factor_diff_pct"]["reference"][f"{s:g}"] = \
            100.0 * (output_factor(ref[s], ref[10.0]) / of_m - 1.0)
        result["output_factor_diff_pct"]["commissioned"][f"{s:g}"] = \
            100.0 * (output_factor(com[s], com[10.0]) / of_m - 1.0)
    fitted = As @ x
    result.update({
        "bases": int(nb), "bases_used": int(used.sum()), "rows": int(As.shape[0]),
        "smooth": float(smooth), "min_sensitivity": float(min_sens),
        "basis_histories": int(n_a), "t_basis_doses_s": t_a,
        "hist_per_field": int(hist_per_field), "hist_measured": int(hist_measured),
        "nnls": {"iters": rep["iters"], "converged": rep["converged"], "t_s": t_fit,
                 "rel_residual": float(np.linalg.norm(fitted - bs) / np.linalg.norm(bs)),
                 "rel_residual_uncommissioned": float(np.linalg.norm(As @ np.ones(nb) - bs)
                                                      / np.linalg.norm(bs))},
        "t_total_s": time.perf_counter() - t_start,
    })
    return result


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--hist-per-basis", type=float, default=1e7)
    ap.add_argument("--hist-per-field", type=float, default=3e9,
                    help="histories per field of the reference and commissioned models")
    ap.add_argument("--hist-measured", type=float, default=1e10,
                    help="histories per field of the measured beam")
    ap.add_argument("--max-iter", type=int, default=300000)
    ap.add_argument("--seed", type=int, default=20150306)
    ap.add_argument("--smooth", type=float, default=0.0,
                    help="weight of the ring-to-ring smoothness term of the fit (0 = Eq. 8 alone)")
    ap.add_argument("--min-sensitivity", type=float, default=0.0,
                    help="fit only bases whose dose column is at least this fraction of the "
                         "median column (0 = every basis some row sees)")
    args = ap.parse_args()

    def log(m):
        print(m, file=sys.stderr, flush=True)

    print(json.dumps(evaluate(args.hist_per_basis, args.hist_per_field, args.hist_measured,
                              args.max_iter, args.seed, smooth=args.smooth, log=log,
                              min_sens=args.min_sensitivity)))


if __name__ == "__main__":
    main()
