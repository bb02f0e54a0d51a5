"""Oracle pins for transport and tally: exact energy conservation, uncollided
transmission exp(-sum mu l) through slabs, telescoping CSDA path length,
index-map tally (Sec. 2.2.2) and replica statistics."""
import math

import numpy as np
import pytest

NE_WATER = 6.02214076e23 * 10.0 / 18.0153


def _ledger_residual(led):
    out = led["jaw"] + led["missed"] + led["invalid"] + led["esc_g"] + led["esc_e"] + led["dep"]
    return (led["src"] - out) / led["src"]


def test_ledger_closes_water(orc, wl):
    W = wl.workload("water60_10x10")
    w, _ = orc.psl_build(W.model)
    plan = orc.plan_build(W.model, w, W.beams, 20000)
    s, s2, led, cnt = orc.run(W.model, plan, W.beams, W.phantom, 11, 2)
    assert abs(_ledger_residual(led)) < 1e-12
    assert led["dep"] == pytest.approx(s.sum(), rel=1e-12)
    assert cnt["hist"] == 40000
    assert cnt["wc_steps"] == cnt["real"]          # homogeneous: every collision is real


def test_ledger_closes_heterogeneous(orc, wl):
    ph = wl.hetero_phantom(5, nx=48, ny=32, nz=48, vox=0.5)
    m = wl.psr_model(5)
    beams = wl.hetero_beams(5, 3)
    w, _ = orc.psl_build(m)
    plan = orc.plan_build(m, w, beams, 20000)
    s, s2, led, cnt = orc.run(m, plan, beams, ph, 12, 1)
    assert abs(_ledger_residual(led)) < 1e-12
    assert cnt["wc_steps"] > cnt["real"]            # virtual collisions in lung
    assert led["missed"] >= 0 and cnt["entered"] > 0


@pytest.mark.parametrize("e", [0.1, 1.0, 4.0])
def test_uncollided_transmission_through_slabs(orc, wl, e):
    """Narrow beam along z through water / lung / bone / water slabs: the
    fraction leaving without a real interaction is exp(-sum_i mu_i l_i)."""
    slabs = [(10, 1.0), (8, 0.26), (4, 1.85), (6, 1.0)]
    ph = wl.slab_phantom(5, 1.0, slabs, 0.5)
    n = 200000
    pos = np.tile([0.01, -0.02, 0.0], (n, 1))
    dirs = np.tile([0.0, 0.0, 1.0], (n, 1))
    edep, led, cnt = orc.transport(ph, 3, np.zeros(n), pos, dirs, np.full(n, e),
                                   np.arange(n, dtype=np.uint64))
    mu_l = sum(NE_WATER * rho * orc.kn_sigma(e) * k * 0.5 for k, rho in slabs)
    p = math.exp(-mu_l)
    frac = cnt["esc_uncollided"] / n
    assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / n)
    assert abs(_ledger_residual(led)) < 1e-12


@pytest.mark.parametrize("rho", [1.0, 1.85])
def test_csda_path_telescopes_to_range(orc, wl, rho):
    """With multiple scattering off, every electron step covers a range
    difference, so the total path of an electron of energy E0 stopped inside a
    uniform medium is R(E0) / rho, and all of E0 is deposited."""
    ph = wl.water_phantom(40, 0.25, rho=rho)
    n = 500
    e0 = np.linspace(0.3, 5.0, n)
    pos = np.tile([0.013, -0.021, 5.0], (n, 1))
    rng = np.random.default_rng(1)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    tp = orc.params(ms=False)
    edep, led, cnt = orc.transport(ph, 5, np.ones(n), pos, d, e0, np.arange(n, dtype=np.uint64),
                                   tparams=tp)
    rho32 = float(np.float32(rho))     # phantom densities are float32
    expect = sum(orc.csda_range(x, 0.2) for x in e0) / rho32
    assert led["e_path"] == pytest.approx(expect, rel=1e-9)
    assert led["dep"] == pytest.approx(e0.sum(), rel=1e-12)
    assert led["esc_e"] == 0.0
    assert cnt["e_boundary"] > 0


def test_index_map_tally_matches_grid(orc, wl):
    W = wl.workload("water60_10x10")
    w, _ = orc.psl_build(W.model)
    bmap = wl.commissioning_basis_map(W.model)
    plan = orc.plan_build(W.model, w, W.beams, 20000, basis_map=bmap)
    imap, n_rows = wl.commissioning_index_map(60, 0.5)
    s, s2, led, cnt = orc.run(W.model, plan, W.beams, W.phantom, 21, 1)
    t, t2, led2, cnt2 = orc.run(W.model, plan, W.beams, W.phantom, 21, 1, index_map=imap,
                                n_rows=n_rows, n_cols=720)
    tab = t.reshape(n_rows, 720)
    sel = np.flatnonzero(imap.ravel())
    rows = imap.ravel()[sel] - 1
    assert np.allclose(tab.sum(axis=1)[rows], s[sel], rtol=1e-12, atol=1e-12)
    assert led2["dep"] == pytest.approx(led["dep"], rel=1e-12)
    assert tab.sum() > 0 and np.count_nonzero(tab.sum(axis=0)) > 50


def test_replica_sigma_scales_inverse_sqrt_n(orc, wl):
    """Replica spread of 5x5x5-voxel block energies falls as 1/sqrt(N)."""
    W = wl.workload("water60_10x10")
    w, _ = orc.psl_build(W.model)
    rel = []
    for n in (5000, 20000):
        plan = orc.plan_build(W.model, w, W.beams, n)
        reps = []
        for r in range(10):
            s, _, _, _ = orc.run(W.model, plan, W.beams, W.phantom, 33, 1, rep0=r)
            reps.append(s.reshape(12, 5, 12, 5, 12, 5).sum(axis=(1, 3, 5)).ravel())
        reps = np.array(reps)
        mean = reps.mean(axis=0)
        sd = reps.std(axis=0, ddof=1)
        hi = mean > 0.5 * mean.max()
        rel.append(np.sqrt(np.mean((sd[hi] / mean[hi]) ** 2)))
    assert rel[0] / rel[1] == pytest.approx(2.0, rel=0.2)


def test_depth_dose_shape(orc, wl):
    W = wl.workload("water60_10x10")
    w, _ = orc.psl_build(W.model)
    plan = orc.plan_build(W.model, w, W.beams, 100000)
    s, s2, led, cnt = orc.run(W.model, plan, W.beams, W.phantom, 44, 2)
    e = s.reshape(60, 60, 60)
    cax = e[:, 28:32, 28:32].sum(axis=(1, 2))
    # attenuation with depth beyond the maximum, and a penumbra: dose outside
    # the field much lower than inside at 10 cm depth
    assert cax[50] < 0.6 * cax.max()
    prof = e[20, 28:32, :].sum(axis=0)
    assert prof[:15].mean() < 0.15 * prof[25:35].mean()


# SI: 1 MeV = 1e6 x 1.602176634e-19 J (exact); a mass of rho V g is rho V 1e-3 kg
GY_PER_MEV_PER_G = 1e6 * 1.602176634e-19 / 1e-3


def test_finalize_closed_form(orc, wl):
    """Dose = mean replica energy (MeV) converted to J over the voxel mass in
    kg, times the model particles per history; sigma = standard error of the
    replica mean (sample standard deviation over sqrt(R))."""
    ph = wl.Phantom(np.array([[[1.0, 0.5, 0.0]]], dtype=np.float32), (0.5, 0.4, 0.3),
                    (0.0, 0.0, 0.0))
    reps = np.array([[1.0, 4.0, 2.0], [2.0, 4.0, 3.0], [3.0, 4.0, 1.0]])
    s, s2 = reps.sum(axis=0), (reps ** 2).sum(axis=0)
    w = 2.5
    dose, sig = orc.finalize(ph, s, s2, 3, w)
    vol = 0.5 * 0.4 * 0.3
    assert dose[0] == pytest.approx(2.0 * GY_PER_MEV_PER_G / (1.0 * vol) * w, rel=1e-14, abs=0)
    assert sig[0] == pytest.approx(math.sqrt(1.0 / 3.0) * GY_PER_MEV_PER_G / vol * w, rel=1e-12,
                                   abs=0)
    assert dose[1] == pytest.approx(4.0 * GY_PER_MEV_PER_G / (0.5 * vol) * w, rel=1e-14, abs=0)
    assert sig[1] == 0.0
    assert dose[2] == 0.0 and sig[2] == 0.0         # no mass, no dose


def test_commissioning_columns_sum_to_open_field_dose(orc, wl):
    """Sec. 2.2.2-2.2.3: with every correction factor at 1 the basis doses add
    up to the dose of the model itself.  The basis columns come from a
    stratified plan (each basis gets the same number of histories, weighted
    by its in-area weight over its count); the open-field dose from the
    Eq. (3) plan through the oracle's finalisation.  Both are normalised
    independently; they must agree row by row within the statistical error."""
    W = wl.workload("water60_10x10")
    imap, n_rows = wl.commissioning_index_map(60, 0.5)
    j = np.arange(W.model.n_ring)
    bmap = np.zeros((3, W.model.n_ebin, W.model.n_ring), dtype=np.uint16)
    for s in range(3):
        bmap[s] = s * 3 + np.minimum(j // 10, 2)[None, :]
    n_cols, n_rep = 9, 8
    w_psl, _ = orc.psl_build(W.model)
    pc = orc.plan_build(W.model, w_psl, W.beams, 0, basis_map=bmap, hist_per_basis=20000)
    n_open = 180000
    po = orc.plan_build(W.model, w_psl, W.beams, n_open)
    sel = np.flatnonzero(imap.ravel())
    rows = imap.ravel()[sel] - 1
    used = pc.group_n > 0
    assert used.sum() >= 6
    # basis columns in Gy per model particle: (energy / n_k) * S_k / (rho V),
    # one replica at a time so that sums over rows get their own spread
    col_w = np.where(used, pc.group_w / np.maximum(pc.group_n, 1), 0.0)
    k = GY_PER_MEV_PER_G * col_w[None, :] / (1.0 * 0.5 ** 3)
    a_r, d_r = [], []
    for r in range(n_rep):
        t, _, _, _ = orc.run(W.model, pc, W.beams, W.phantom, 61, 1, rep0=r, index_map=imap,
                             n_rows=n_rows, n_cols=n_cols)
        a_r.append((k * t.reshape(n_rows, n_cols)).sum(axis=1))
        e, e2, _, _ = orc.run(W.model, po, W.beams, W.phantom, 62, 1, rep0=r)
        dose, _ = orc.finalize(W.phantom, e, e2, 1, po.w.sum() / n_open)
        d_rows = np.zeros(n_rows)
        d_rows[rows] = dose[sel]
        d_r.append(d_rows)
    a_r, d_r = np.array(a_r), np.array(d_r)
    a, d = a_r.mean(axis=0), d_r.mean(axis=0)
    sa, sd = a_r.std(axis=0, ddof=1) / math.sqrt(n_rep), d_r.std(axis=0, ddof=1) / math.sqrt(n_rep)
    hi = d > 0.2 * d.max()
    assert hi.sum() > 80
    z = (a[hi] - d[hi]) / np.sqrt(sa[hi] ** 2 + sd[hi] ** 2)
    assert np.mean(np.abs(z) < 3) > 0.95
    assert abs(np.mean(z)) < 0.5

    def z_sum(scale):
        """The sum over the compared rows against its replica spread."""
        sa_, sd_ = (a_r[:, hi] * scale).sum(axis=1), d_r[:, hi].sum(axis=1)
        diff = sa_ - sd_
        return diff.mean() / (diff.std(ddof=1) / math.sqrt(n_rep))

    assert abs(z_sum(1.0)) < 3
    # a dose scaled by a misplaced model-weight factor (here the primary
    # sub-source's share of the weight) fails the same comparisons
    w_frac = pc.group_w[:3].sum() / pc.group_w.sum()
    assert w_frac < 0.9
    z_bad = (a[hi] * w_frac - d[hi]) / np.sqrt(sa[hi] ** 2 + sd[hi] ** 2)
    assert abs(np.mean(z_bad)) > 0.5
    assert abs(z_sum(w_frac)) > 3
