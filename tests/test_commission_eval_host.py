"""Host side of the paper-shaped commissioning: the basis layout (one unit
per photon PSR, one per electron energy bin), the curve rows of the index
map, and the comparison metrics on curves whose answers are known in closed
form (a shifted edge has a DTA equal to the shift; a scaled depth dose has
RMS and maximum differences equal to the scale)."""
import math

import numpy as np
import pytest

from paper_1503_01725_amd import commission_eval as ce
from paper_1503_01725_amd import workloads as wl


def test_basis_map_units():
    m = wl.psr_model(3, n_ebin=6, n_ring=5, n_psl=10)
    bm = ce.basis_map(m).astype(int)
    nb = ce.n_basis(m)
    assert bm.shape == (3, 6, 5) and nb == 2 * 6 * 5 + 6
    photon = bm[:2].ravel()
    assert len(set(photon.tolist())) == photon.size          # one per photon PSR
    for b in range(6):
        assert len(set(bm[2, b].tolist())) == 1                # one per electron bin
    assert sorted(set(bm.ravel().tolist())) == list(range(nb))
    x = np.arange(1, nb + 1, dtype=float)
    c = ce.corrected_model(m, x)
    assert np.allclose(c.w_psr, m.w_psr * x[bm])


def test_wide_model_has_fewer_bases_than_rows():
    m = ce.wide_model(5)
    _, n_rows, _ = ce.index_map()
    assert ce.n_basis(m) == 2 * 10 * 30 + 10
    assert ce.n_basis(m) < 2 * (1 + 2 * len(ce.DEPTHS)) * ce.N_VOX
    assert m.n_ring * m.ring_dr >= 20.0 * math.sqrt(2.0)   # the 40 x 40 corner at the plane


def test_dta_window_and_surface():
    pos = np.array([0.25, 0.75, 1.25, 1.75])
    meas = np.array([0.6, 0.8, 1.0, 0.98])
    calc = np.array([0.7, 0.9, 1.0, 0.98])         # 0.1 higher on the rise (slope 0.4 / cm)
    t = ce.dta(pos, meas, calc, np.array([True, True, False, False]))
    assert np.allclose(t, 0.25)
    far = ce.dta(pos, meas, calc + 5.0, np.array([True, False, False, False]), window=1.5)
    assert far[0] == 1.5


def test_measured_beam_is_a_smooth_reweighting():
    m = ce.wide_model(5)
    mm = ce.measured_model(m)
    r = mm.w_psr / m.w_psr
    assert r.shape == m.w_psr.shape and np.all(r > 0.5) and np.all(r < 1.75)
    assert not np.allclose(r[2], r[2][:, :1])     # electrons vary with the ring too
    assert np.allclose(ce.measured_model(m, 0.0).w_psr, m.w_psr)


def test_index_map_rows_follow_the_curves():
    n, vox = 48, 0.5
    sel_names = [c for c, _, _ in ce.curve_voxels(n, vox)]
    assert sel_names[0] == "pdd" and len(sel_names) == 1 + 2 * len(ce.DEPTHS)
    grid = np.arange(n ** 3, dtype=float).reshape(n, n, n)
    cur = ce.curves_of_grid(grid, n, vox)
    c = n // 2
    assert np.array_equal(cur["pdd"], grid[:, c, c])
    k = int(math.floor(10.0 / vox))
    assert np.array_equal(cur["inline_10"], grid[k, :, c])
    assert np.array_equal(cur["crossline_10"], grid[k, c, :])


def test_index_map_full_size():
    imap, n_rows, rows = ce.index_map()
    grid = np.random.default_rng(1).random(imap.shape)
    flat = np.zeros(n_rows)
    sel = imap > 0
    flat[imap[sel] - 1] = grid[sel]
    cur = ce.curves_of_grid(grid)
    for name, r in rows.items():
        assert np.array_equal(flat[r], cur[name]), name


def test_dta_of_a_shifted_edge():
    pos = np.linspace(-10, 10, 401)
    edge = lambda x: 1.0 / (1.0 + np.exp(x / 0.3))
    meas, calc = edge(pos), edge(pos - 0.2)        # calc shifted by +0.2 cm
    sel = (meas > 0.2) & (meas < 0.8)
    t = ce.dta(pos, meas, calc, sel)
    assert np.allclose(t, 0.2, atol=2e-3)
    assert np.all(ce.dta(pos, meas, meas, sel) < 1e-9)


def test_depth_dose_rms_and_max_of_a_scaled_curve():
    z = np.linspace(0.25, 31.75, 64)
    meas = np.where(z < 1.5, 0.5 + z / 3.0, np.exp(-0.05 * (z - 1.5)))
    calc = meas * 1.02
    m = ce.depth_dose_metrics(z, meas, calc)
    kmax = int(np.argmax(meas))
    after = meas[kmax:-2]
    expect = 2.0 * after / meas.max()
    assert m["rms_pct"] == pytest.approx(float(np.sqrt(np.mean(expect ** 2))), rel=1e-12)
    assert m["max_pct"] == pytest.approx(2.0, rel=1e-12)


def test_profile_regions():
    pos = np.linspace(-20, 20, 161)
    prof = 1.0 / (1.0 + np.exp((np.abs(pos) - 5.0) / 0.4))
    m = ce.profile_metrics(pos, prof, prof * 1.01)
    assert m["inner_max_pct"] == pytest.approx(1.0 * prof[prof / prof[80] >= 0.8].max() / prof[80],
                                               rel=1e-9)
    assert m["penumbra_dta_max_cm"] < 0.1


def test_smoothness_rows_pair_neighbouring_photon_rings():
    from paper_1503_01725_amd import commission_eval as ce
    m = ce.wide_model(3)
    D = ce.smoothness_rows(m)
    assert D.shape == (2 * m.n_ebin * (m.n_ring - 1), ce.n_basis(m))
    bm = ce.basis_map(m).astype(np.int64)
    electron = set(bm[2].ravel().tolist())
    for row in D:
        i, j = np.flatnonzero(row == 1.0), np.flatnonzero(row == -1.0)
        assert len(i) == 1 and len(j) == 1 and np.count_nonzero(row) == 2
        s, b, r = np.argwhere(bm[:2] == i[0])[0]
        assert bm[s, b, r + 1] == j[0]
        assert i[0] not in electron and j[0] not in electron
    # a constant correction is not penalised
    assert np.allclose(D @ np.full(D.shape[1], 1.7), 0.0)


def test_scaled_system_adds_the_smoothness_term():
    """|A1 y - b1|^2 = |A x - b|^2 / scale^2 + smooth |D x|^2 with y = x * cn on
    the used bases and x = 1 on the unused ones."""
    from paper_1503_01725_amd import commission_eval as ce
    rng = np.random.default_rng(11)
    A = rng.uniform(0, 1, (30, 12))
    A[:, [3, 7, 8]] = 0.0                      # bases no row sees
    b = rng.uniform(0, 2, 30)
    D = np.zeros((11, 12))
    for k in range(11):
        D[k, k], D[k, k + 1] = 1.0, -1.0
    for lam in (0.0, 0.3):
        A1, b1, used, cn, scale = ce.scaled_system(A, b, D, lam)
        x = rng.uniform(0, 2, 12)
        x[~used] = 1.0
        y = x[used] * cn
        lhs = np.sum((A1 @ y - b1) ** 2)
        rhs = np.sum((A @ x - b) ** 2) / scale ** 2 + lam * np.sum((D @ x) ** 2)
        assert lhs == pytest.approx(rhs, rel=1e-12)
    assert A1.shape[0] == 30 + 10                  # the row of unused bases 7 and 8 is dropped


def test_scaled_system_leaves_weakly_seen_bases_at_one():
    """With a sensitivity threshold, bases whose dose column falls below it
    are not fitted: they keep the factor 1, their dose moves to the
    right-hand side, and |A1 y - b1|^2 = |A x - b|^2 / scale^2 still holds."""
    from paper_1503_01725_amd import commission_eval as ce
    rng = np.random.default_rng(12)
    A = rng.uniform(0, 1, (30, 12))
    A[:, 3] = 0.0                              # a basis no row sees
    A[:, 5] *= 1e-6                            # a basis the rows barely see
    b = rng.uniform(0, 2, 30)
    A1, b1, used, cn, scale = ce.scaled_system(A, b, min_sens=1e-3)
    assert not used[3] and not used[5] and used.sum() == 10
    x = rng.uniform(0, 2, 12)
    x[~used] = 1.0
    y = x[used] * cn
    lhs = np.sum((A1 @ y - b1) ** 2)
    assert lhs == pytest.approx(np.sum((A @ x - b) ** 2) / scale ** 2, rel=1e-12)
    A1_0, b1_0, used_0, _, _ = ce.scaled_system(A, b)
    assert used_0[5] and not used_0[3] and used_0.sum() == 11
