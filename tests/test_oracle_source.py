"""Oracle pins for the source side: PSR->PSL conversion (Sec. 2.1.1, Eqs. 1-2),
sampling areas (Sec. 2.1.2, Fig. 3), Eq. (3) counts and steps S3-S5."""
import math

import numpy as np
import pytest
from scipy import stats

import dataclasses


def _centres(m):
    c = m.psl_x0 + (np.arange(m.n_psl) + 0.5) * m.psl_dx
    return np.sqrt(c[None, :] ** 2 + c[:, None] ** 2)   # [iy][ix]


def test_psl_uniform_closed_form(orc, wl):
    """With W_R proportional to ring area (no noise), the interpolated ring
    weight is linear in r, so Eq. (2) gives exactly uniform PSL weights for
    centres between the first and last ring centre, W_last*r_last/r beyond it,
    and 0 outside the model radius."""
    m = wl.psr_model(3, noise=False, simple_scatter=True)
    w, total = orc.psl_build(m)
    r = _centres(m)
    r_first, r_last, r_out = 0.5 * m.ring_dr, (m.n_ring - 0.5) * m.ring_dr, m.n_ring * m.ring_dr
    inner = (r >= r_first) & (r <= r_last)
    tail = (r > r_last) & (r <= r_out)
    outside = r > r_out
    assert inner.sum() > 2700 and tail.sum() > 0 and outside.sum() > 0
    for s in range(3):
        for b in range(m.n_ebin):
            plane = w[s, b]
            ref = plane[inner].mean()
            if ref == 0.0:
                assert np.all(plane == 0.0)
                continue
            assert np.allclose(plane[inner], ref, rtol=1e-12, atol=0)
            assert np.allclose(plane[tail], ref * r_last / r[tail], rtol=1e-12, atol=0)
            assert np.all(plane[outside] == 0.0)
    assert abs(w.sum() - 1.0) < w.size * 2.3e-16   # sequential-sum rounding bound


def test_psl_matches_library_interpolation(orc, wl):
    """General noisy model: steps 1-4 of Sec. 2.1.1 with numpy's piecewise-linear
    interpolation (clamped at both ends) as the interpolation step."""
    m = wl.psr_model(7)
    w, total = orc.psl_build(m)
    r = _centres(m)
    rc = (np.arange(m.n_ring) + 0.5) * m.ring_dr
    ref = np.zeros_like(w)
    for s in range(3):
        for b in range(m.n_ebin):
            wt = np.interp(r, rc, m.w_psr[s, b])
            wt[r > m.n_ring * m.ring_dr] = 0.0
            ref[s, b] = wt / (2 * math.pi * r)
    ref /= ref.sum()
    assert np.allclose(w, ref, rtol=1e-11, atol=0)
    # continuum identity (Eq. 1), noise-free model: the PSL weights whose
    # centres fall in ring j add up to about W_R,j * dr / (dx^2 * S); only the
    # discretisation of the ring by PSL squares separates them
    m0 = wl.psr_model(7, noise=False)
    w0, total0 = orc.psl_build(m0)
    idx = np.floor(r / m.ring_dr).astype(int)
    for s, b in ((0, 10), (1, 3), (2, 20)):
        ring_sum = np.array([w0[s, b][idx == j].sum() for j in range(m.n_ring)])
        expv = m0.w_psr[s, b] * m.ring_dr / (m.psl_dx ** 2 * total0)
        # annuli of 5 rings each (lattice-point counting noise averages out)
        rel = ring_sum[5:25].reshape(4, 5).sum(1) / expv[5:25].reshape(4, 5).sum(1)
        assert np.all(np.abs(rel - 1) < 0.05), rel


def test_scatter_cdf(orc, wl):
    m = wl.psr_model(5)
    P = orc.scatter_cdf(m)
    c = m.sc_c
    ref = np.cumsum(c, axis=-1) / c.sum(axis=-1, keepdims=True)
    assert np.allclose(P[..., :-1], ref[..., :-1], rtol=1e-15, atol=1e-16)
    assert np.all(P[..., -1] == 1.0)
    assert np.all(np.diff(P, axis=-1) > 0)


def test_sampling_box_hand_values(orc, wl):
    """10x10 field: primary area = jaw opening + shadow of a 4-sigma focal spot
    through the jaw edge (Y: 4*0.1*72/28 cm, X: 4*0.1*63/37 cm), expanded to
    whole PSLs with positive-area overlap."""
    m = wl.psr_model(1)
    b = wl.square_beam(10.0)
    # y: [-6.02857, 6.02857] -> iy 17..42 ; x: [-5.68108, 5.68108] -> ix 18..41
    assert orc.sampling_box(m, b, 0) == (18, 41, 17, 42)
    # no focal spot: the opening itself; PSLs that only touch an edge are excluded
    m0 = dataclasses.replace(m, sigma_spot=0.0)
    assert orc.sampling_box(m0, b, 0) == (20, 39, 20, 39)
    b2 = wl.Beam(-2.2, 3.0, -1.0, 0.75)
    # x: floor(12.8/0.5)=25 .. ceil(36/0.5)-1=35 ; y: 28 .. ceil(31.5)-1=31
    assert orc.sampling_box(m0, b2, 0) == (25, 35, 28, 31)


def test_eq3_counts_exact_totals(orc, wl):
    W = wl.workload("hetero256_5beam")
    w, _ = orc.psl_build(W.model)
    for n in (1, 7, 10 ** 5, 123456789, 2 * 10 ** 8):
        plan = orc.plan_build(W.model, w, W.beams, n)
        cnt = plan.counts.astype(np.float64)
        assert int(plan.counts.sum()) == n
        q = np.array([round(x * 2.0 ** 40) for x in plan.w], dtype=np.float64)
        share = n * q / q.sum()
        assert np.all(np.abs(cnt - share) < 1.0)
        assert np.all((cnt == np.floor(share)) | (cnt == np.ceil(share)))
    # list order: beam, sub-source, energy bin, iy, ix (locations inner)
    key = (((plan.beam.astype(np.int64) * 3 + plan.stype) * 24 + plan.ebin) * 60
           + plan.iy) * 60 + plan.ix
    assert np.all(np.diff(key) > 0)
    # group weight = sum of in-area weights over all beams (Eq. 3 denominator)
    assert plan.group_w[0] == pytest.approx(plan.w.sum(), rel=1e-14)


def test_stratified_counts(orc, wl):
    W = wl.workload("commission60")
    w, _ = orc.psl_build(W.model)
    bmap = W.extra["basis_map"]
    plan = orc.plan_build(W.model, w, W.beams, 0, basis_map=bmap, hist_per_basis=1000)
    tags, first = np.unique(plan.tag, return_index=True)
    assert np.all(np.diff(plan.tag) >= 0)
    per_tag = np.bincount(plan.tag, weights=plan.counts.astype(np.float64),
                          minlength=4 * 720)
    assert np.all(per_tag[tags] == 1000)
    assert plan.n_hist == 1000 * len(tags)
    for t in tags[::97]:
        sel = plan.tag == t
        assert plan.group_w[t] == pytest.approx(plan.w[sel].sum(), rel=1e-13)
        # basis ids follow the map at the PSL centre ring
        beam = t // 720
        k = t % 720
        c = W.model.psl_x0 + (np.array([plan.ix[sel], plan.iy[sel]]) + 0.5) * W.model.psl_dx
        ring = np.minimum(np.floor(np.hypot(c[0], c[1]) / W.model.ring_dr).astype(int), 29)
        assert np.all(bmap[plan.stype[sel], plan.ebin[sel], ring] == k)
        assert np.all(plan.beam[sel] == beam)


def _full_plane_plan(orc, model, w_psl, per_weight=2.0e7):
    """A plan over every PSL of the plane (no sampling area), built directly."""
    s, b, iy, ix = np.nonzero(w_psl > 0)
    order = np.lexsort((ix, iy, b, s))
    s, b, iy, ix = s[order], b[order], iy[order], ix[order]
    wv = w_psl[s, b, iy, ix]
    cnt = np.maximum(1, np.round(wv * per_weight)).astype(np.uint64)
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    return orc.Plan(i32(np.zeros_like(s)), i32(s), i32(b), i32(ix), i32(iy), i32(np.zeros_like(s)),
                    wv, np.cumsum(cnt).astype(np.uint64), np.zeros(1), np.zeros(1, np.uint64),
                    int(cnt.sum()))


@pytest.mark.parametrize("narrow", [False, True])
@pytest.mark.parametrize("field", [(10.0, 10.0), (4.0, 12.0)])
def test_sampling_area_brute_force(orc, wl, field, narrow):
    """Sample the whole plane with no area limit and apply the jaws: at most
    0.5% of the surviving weight may come from PSLs outside the sampling area.
    The narrow model has direction spreads small enough for the scatter and
    electron areas to be proper subsets of the plane."""
    if narrow:
        m = wl.psr_model(9, scatter_sigma_cm=0.3, sig_e=0.01)
    else:
        m = wl.psr_model(9)
    w, _ = orc.psl_build(m)
    beam = wl.Beam(-field[0] / 2, field[0] / 2, -field[1] / 2, field[1] / 2)
    plan = _full_plane_plan(orc, m, w)
    ph = wl.water_phantom(60, 0.5)
    rec = orc.sample(m, plan, [beam], ph, 77, 0, plan.n_hist)
    ok = rec["status"] != 1
    n_sub = 0
    for s in range(3):
        box = orc.sampling_box(m, beam, s)
        n_sub += (box[1] - box[0] + 1) * (box[3] - box[2] + 1) < m.n_psl ** 2
        sel = ok & (rec["stype"] == s)
        inside = ((rec["ix"] >= box[0]) & (rec["ix"] <= box[1]) &
                  (rec["iy"] >= box[2]) & (rec["iy"] <= box[3]))
        wt = plan.w[rec["j"]] / plan.counts[rec["j"]].astype(np.float64)
        out_frac = wt[sel & ~inside].sum() / wt[sel].sum()
        assert out_frac <= 0.005, (s, out_frac)
    assert n_sub == 3 if narrow else n_sub >= 1


@pytest.fixture(scope="module")
def sampled(orc, wl):
    W = wl.workload("water60_10x10")
    w, _ = orc.psl_build(W.model)
    plan = orc.plan_build(W.model, w, W.beams, 200000)
    rec = orc.sample(W.model, plan, W.beams, W.phantom, 4242, 0, plan.n_hist)
    return W, plan, rec


def test_history_to_psl_mapping_exact(sampled):
    W, plan, rec = sampled
    assert np.array_equal(np.bincount(rec["j"], minlength=len(plan.cum)),
                          plan.counts.astype(np.int64))


def test_position_and_energy_uniform_within_psl(sampled):
    W, plan, rec = sampled
    m = W.model
    fx = (rec["xb"] - (m.psl_x0 + rec["ix"] * m.psl_dx)) / m.psl_dx
    fy = (rec["yb"] - (m.psl_x0 + rec["iy"] * m.psl_dx)) / m.psl_dx
    fe = (rec["e"] - (m.e_lo + rec["ebin"] * m.e_width)) / m.e_width
    for f in (fx, fy, fe):
        assert f.min() >= 0 and f.max() < 1
        assert stats.kstest(f, "uniform").pvalue > 1e-3


def test_primary_back_trace_hits_focal_spot(sampled):
    """Eq. (5) rotated by theta: the primary ray traced back to the target plane
    lands on the sampled focal-spot point rotated into the global frame."""
    W, plan, rec = sampled
    m = W.model
    p = rec[rec["stype"] == 0]
    t = (m.z_plane - m.z_target) / p["wb"]
    xt = p["xb"] - t * p["ub"]
    yt = p["yb"] - t * p["vb"]
    r = np.hypot(p["xb"], p["yb"])
    c, s = p["xb"] / r, p["yb"] / r
    xs = c * p["xs"] - s * p["ys"]
    ys = s * p["xs"] + c * p["ys"]
    assert np.max(np.abs(xt - xs)) < 1e-9 and np.max(np.abs(yt - ys)) < 1e-9
    # focal spot is a 2D Gaussian with sigma_s (Eq. 4)
    assert stats.kstest(p["xs"] / m.sigma_spot, "norm").pvalue > 1e-3
    assert stats.kstest(p["ys"] / m.sigma_spot, "norm").pvalue > 1e-3


def test_scatter_mixture_and_angles(sampled):
    """Eq. (6): component frequencies follow c_{i,k}; within a component
    (alpha - mu)/sigma_alpha and beta/sigma_beta are standard normal; the local
    direction has alpha = atan(u/w), beta = atan(v/w)."""
    W, plan, rec = sampled
    m = W.model
    sc = rec[rec["stype"] == 1]
    r = np.hypot(sc["xb"], sc["yb"])
    ring = np.minimum(np.floor(r / m.ring_dr).astype(int), m.n_ring - 1)
    c = m.sc_c[sc["ebin"], ring]
    pk = c / c.sum(axis=1, keepdims=True)
    obs = np.bincount(sc["k"], minlength=3)
    expv = pk.sum(axis=0)
    chi2 = ((obs - expv) ** 2 / expv).sum()
    assert chi2 < 13.8   # 2 dof, p = 1e-3
    mu = m.sc_mu[sc["ebin"], ring, sc["k"]]
    sa = m.sc_sa[sc["ebin"], ring, sc["k"]]
    sb = m.sc_sb[sc["ebin"], ring, sc["k"]]
    assert stats.kstest((sc["alpha"] - mu) / sa, "norm").pvalue > 1e-3
    assert stats.kstest(sc["beta"] / sb, "norm").pvalue > 1e-3
    # undo the rotation by theta and recover the angles
    cth, sth = sc["xb"] / r, sc["yb"] / r
    ul = cth * sc["ub"] + sth * sc["vb"]
    vl = -sth * sc["ub"] + cth * sc["vb"]
    assert np.allclose(np.arctan(ul / sc["wb"]), sc["alpha"], atol=1e-12)
    assert np.allclose(np.arctan(vl / sc["wb"]), sc["beta"], atol=1e-12)


def test_electron_angles(sampled):
    W, plan, rec = sampled
    el = rec[rec["stype"] == 2]
    assert len(el) > 1000
    assert stats.kstest(el["alpha"] / W.model.sig_ea, "norm").pvalue > 1e-3
    assert stats.kstest(el["beta"] / W.model.sig_eb, "norm").pvalue > 1e-3


def test_jaw_rejection_brute_force(sampled):
    """Independent jaw test: trace every particle to each jaw plane and compare
    with the focused jaw opening there."""
    W, plan, rec = sampled
    m, b = W.model, W.beams[0]
    ok = rec["status"] != 3
    r = rec[ok]
    zy, zx = m.z_jaw_y, m.z_jaw_x
    yj = r["yb"] + r["vb"] / r["wb"] * zy
    xj = r["xb"] + r["ub"] / r["wb"] * zx
    fy = (zy + 100.0) / 100.0
    fx = (zx + 100.0) / 100.0
    passed = (yj >= b.y1 * fy) & (yj <= b.y2 * fy) & (xj >= b.x1 * fx) & (xj <= b.x2 * fx)
    assert np.array_equal(passed, r["status"] != 1)
    # water cube top face is the plane: accepted rays enter at z = 0 (t = 0)
    acc = r[r["status"] == 0]
    assert np.allclose(acc["z"], 0.0, atol=1e-12)


def test_radial_histogram_over_whole_plane(orc, wl):
    """Sampled radius over the whole plane against the exact expectation from
    the PSL squares: counts per annulus = sum over PSLs of n_PSL * (area of the
    square inside the annulus) / (square area), the areas by fine midpoint
    quadrature."""
    m = wl.psr_model(2)
    w, _ = orc.psl_build(m)
    w1 = w.copy()
    w1[1:] = 0.0
    w1[0, :3] = w[0, :3]
    w1[0, 3:] = 0.0
    plan = _full_plane_plan(orc, m, w1, per_weight=3.0e6 / w1.sum())
    big = wl.water_phantom(60, 0.5)
    rec = orc.sample(m, plan, [wl.square_beam(60.0)], big, 31, 0, plan.n_hist)
    r = np.hypot(rec["xb"], rec["yb"])
    edges = np.linspace(0, 15 * math.sqrt(2), 43)
    obs = np.histogram(r, bins=edges)[0].astype(float)
    # expected: per PSL location, the number of histories, spread by area
    n_loc = np.zeros((m.n_psl, m.n_psl))
    np.add.at(n_loc, (plan.iy, plan.ix), plan.counts.astype(float))
    q = 40
    f = (np.arange(q) + 0.5) / q
    expv = np.zeros(len(edges) - 1)
    for iy in range(m.n_psl):
        for ix in range(m.n_psl):
            if n_loc[iy, ix] == 0:
                continue
            xs = m.psl_x0 + (ix + f) * m.psl_dx
            ys = m.psl_x0 + (iy + f) * m.psl_dx
            rr = np.hypot(xs[None, :], ys[:, None]).ravel()
            expv += n_loc[iy, ix] * np.histogram(rr, bins=edges)[0] / rr.size
    keep = expv > 50
    chi2 = ((obs[keep] - expv[keep]) ** 2 / expv[keep]).sum()
    dof = keep.sum() - 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof) + 0.002 * expv[keep].sum() / 100
