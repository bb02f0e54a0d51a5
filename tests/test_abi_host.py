"""C-ABI checks that need no GPU: every symbol of include/psl.h is exported,
and the host set-up calls (psl_build, psl_plan_create, batching) agree with
the oracle bit for bit."""
import ctypes as C

import numpy as np
import pytest


def test_library_exports_every_declared_symbol(N):
    names = N.exported_symbols()
    assert {"psl_build", "sample_batch", "transport_batch", "tally_dose",
            "commission_nnls"} <= set(names)
    L = N.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


class _Host:
    """Host-only use of the ABI (no torch / device memory)."""

    def __init__(self, N, m):
        self.N = N
        self.keep = [np.ascontiguousarray(a, dtype=np.float64)
                     for a in (m.w_psr, m.sc_c, m.sc_mu, m.sc_sa, m.sc_sb)]
        ptr = [a.ctypes.data_as(N.dp) for a in self.keep]
        self.desc = N.psl_psr_desc(m.n_ebin, m.n_ring, m.n_comp, m.n_psl, m.e_lo, m.e_width,
                                   m.ring_dr, m.psl_x0, m.psl_dx, m.z_target, m.z_plane,
                                   m.z_scatter, m.z_jaw_y, m.z_jaw_x, m.sigma_spot, m.sig_ea,
                                   m.sig_eb, *ptr)
        self.h = N.psl_build(self.desc)
        self.m = m

    def weights(self):
        out = np.zeros((3, self.m.n_ebin, self.m.n_psl, self.m.n_psl))
        self.N.check(self.N.lib().psl_model_weights(self.h, out.ctypes.data_as(self.N.dp)))
        return out

    def plan(self, beams, n_hist, basis_map=None, hist_per_basis=0):
        N = self.N
        arr = (N.psl_beam * len(beams))()
        for i, b in enumerate(beams):
            arr[i] = N.psl_beam(b.x1, b.x2, b.y1, b.y2, b.gantry_deg, b.couch_deg,
                                (C.c_double * 3)(*b.iso))
        bm = None if basis_map is None else np.ascontiguousarray(basis_map, dtype=np.uint16)
        p = N.psl_plan_create(self.h, arr, n_hist, 1,
                              None if bm is None else bm.ctypes.data_as(N.u16p), hist_per_basis)
        info = N.psl_plan_info()
        N.check(N.lib().psl_plan_get_info(p, C.byref(info)))
        n = info.n_list
        ints = [np.zeros(n, dtype=np.int32) for _ in range(6)]
        w = np.zeros(n)
        cum = np.zeros(n, dtype=np.uint64)
        N.check(N.lib().psl_plan_list(p, *[a.ctypes.data_as(N.i32p) for a in ints],
                                      w.ctypes.data_as(N.dp), cum.ctypes.data_as(N.u64p)))
        boxes = np.zeros((len(beams), 3, 4), dtype=np.int32)
        N.check(N.lib().psl_plan_boxes(p, boxes.ctypes.data_as(N.i32p)))
        cw = np.zeros(info.n_cols)
        N.check(N.lib().psl_plan_col_weight(p, cw.ctypes.data_as(N.dp)))
        return p, info, ints, w, cum, boxes, cw


@pytest.mark.parametrize("seed,noise", [(1, True), (2, False), (3, True)])
def test_psl_build_bit_exact(N, orc, wl, seed, noise):
    m = wl.psr_model(seed, noise=noise)
    lib_w = _Host(N, m).weights()
    ref, _ = orc.psl_build(m)
    assert np.array_equal(lib_w, ref)


@pytest.mark.parametrize("name", ["water60_10x10", "hetero256_5beam", "water128_20"])
def test_plan_bit_exact(N, orc, wl, name):
    W = wl.workload(name)
    H = _Host(N, W.model)
    p, info, ints, w, cum, boxes, cw = H.plan(W.beams, W.n_hist)
    ref_w, _ = orc.psl_build(W.model)
    ref = orc.plan_build(W.model, ref_w, W.beams, W.n_hist)
    for a, b in zip(ints, (ref.beam, ref.stype, ref.ebin, ref.ix, ref.iy, ref.tag)):
        assert np.array_equal(a, b)
    assert np.array_equal(w, ref.w)
    assert np.array_equal(cum, ref.cum)
    assert info.n_hist == W.n_hist
    assert info.s_area == ref.group_w[0]
    assert np.all(cw == ref.group_w[0] / W.n_hist)
    for bi, b in enumerate(W.beams):
        for s in range(3):
            assert tuple(boxes[bi, s]) == orc.sampling_box(W.model, b, s)
    N.lib().psl_plan_free(p)


def test_commissioning_plan_bit_exact(N, orc, wl):
    W = wl.workload("commission60")
    H = _Host(N, W.model)
    bm = W.extra["basis_map"]
    p, info, ints, w, cum, boxes, cw = H.plan(W.beams, 0, bm, 1000)
    ref_w, _ = orc.psl_build(W.model)
    ref = orc.plan_build(W.model, ref_w, W.beams, 0, basis_map=bm, hist_per_basis=1000)
    assert np.array_equal(ints[5], ref.tag)
    assert np.array_equal(cum, ref.cum)
    used = ref.group_n > 0
    assert info.n_cols == 4 * 720
    assert np.array_equal(cw[used], ref.group_w[used] / 1000.0)
    N.lib().psl_plan_free(p)


@pytest.mark.parametrize("max_batch,band", [(131072, 1), (1000, 3), (7, 24)])
def test_batching_partitions_histories(N, wl, max_batch, band):
    W = wl.workload("hetero256_5beam")
    H = _Host(N, W.model)
    p, info, ints, w, cum, boxes, cw = H.plan(W.beams, 200000)
    nb = C.c_int64()
    N.check(N.lib().psl_plan_set_batching(p, max_batch, band, C.byref(nb)))
    beam, stype, ebin = ints[0], ints[1], ints[2]
    h = 0
    for i in range(nb.value):
        b = N.psl_batch()
        N.check(N.lib().psl_plan_get_batch(p, i, C.byref(b)))
        assert b.h0 == h and 1 <= b.n <= max_batch
        j0 = np.searchsorted(cum, b.h0, side="right")
        j1 = np.searchsorted(cum, b.h0 + b.n - 1, side="right")
        assert np.all(beam[j0:j1 + 1] == b.beam) and np.all(stype[j0:j1 + 1] == b.stype)
        assert np.all(ebin[j0:j1 + 1] // band == b.band)
        h += b.n
    assert h == info.n_hist
    N.lib().psl_plan_free(p)


def test_bad_arguments_report_einval(N, wl):
    m = wl.psr_model(1)
    H = _Host(N, m)
    out = C.c_void_p()
    bad = (N.psl_beam * 1)(N.psl_beam(5, -5, -5, 5, 0, 0, (C.c_double * 3)(0, 0, 0)))
    rc = N.lib().psl_plan_create(H.h, bad, 1, 100, 1, None, 0, C.byref(out))
    assert rc == N.PSL_EINVAL
    assert b"x1 < x2" in N.lib().psl_last_error()
    rc = N.lib().psl_build(None, C.byref(out))
    assert rc == N.PSL_EINVAL
