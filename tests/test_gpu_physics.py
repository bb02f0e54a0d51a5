"""GPU parity of the optional photon processes (photoelectric absorption,
Rayleigh scattering, pair production with positron annihilation) against the
oracle.  Both sides draw the same Philox streams per particle; the GPU reads
its cross-sections and the Rayleigh angle from FP32 tables where the oracle
evaluates the formulas in FP64, so a process choice or a Rayleigh angle can
differ where a uniform falls within table accuracy of a boundary; after
that the two trajectories are independent samples of the same physics.  The
bar is the plain method's: integral dose within 0.1 %, >= 95 % of voxels
above 10 % of Dmax within 2 sigma, the event counts within their Poisson
spread, and the ledger closed."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LEDGER_OUT = ("jaw", "missed", "invalid", "esc_g", "esc_e", "dep")


def _closure(led):
    return (led["src"] - sum(led[k] for k in LEDGER_OUT)) / led["src"]


def _counts_agree(a, b, rel=0.01):
    """Counts of the same histories' events: within 5 Poisson sigma plus a
    relative allowance for trajectories that part after a tipped decision."""
    return abs(a - b) <= 5.0 * math.sqrt(max(b, 1.0)) + rel * b


def _agreement(d1, s1, d2, s2):
    hi = d2 > 0.1 * d2.max()
    sd = np.sqrt(s1 ** 2 + s2 ** 2)
    return (np.abs(d1 - d2) < 2 * sd)[hi].mean(), hi.sum()


@pytest.mark.parametrize("physics", [1, 2, 4, 7, 8, 16, 31],
                         ids=["photo", "rayleigh", "pair", "photons", "delta", "brem", "all"])
def test_dose_with_process_matches_oracle(eng, orc, wl, physics):
    """The 6 MV-like source on the 60^3 water phantom (1e5 histories in 10
    replicas) with each optional process switched on, and all together."""
    import torch
    W = wl.workload("water60_10x10")
    n_hist, seed = 10000, 781
    print(f"[physics parity] oracle water60_10x10 physics={physics}", flush=True)
    ref_w, _ = orc.psl_build(W.model)
    op = orc.plan_build(W.model, ref_w, W.beams, n_hist)
    s_r, s2_r, led_r, cnt_r = orc.run(W.model, op, W.beams, W.phantom, seed, W.n_replica,
                                      tparams=orc.params(physics=physics))
    d_r, sg_r = orc.finalize(W.phantom, s_r, s2_r, W.n_replica, op.group_w[0] / n_hist)
    print(f"[physics parity] gpu physics={physics}", flush=True)
    model = eng.Model(W.model)
    plan = eng.Plan(model, W.beams, n_hist, n_replica=W.n_replica)
    ph = eng.Phantom(W.phantom)
    tally = eng.Tally(ph)
    eng.run_plan_eager(plan, ph, tally, eng.transport_params(physics=physics), seed)
    dose, sig = tally.finalize(plan)
    torch.cuda.synchronize()
    led, cnt = tally.stats()
    d, sg = dose.cpu().numpy().ravel(), sig.cpu().numpy().ravel()
    print(f"[physics parity] dep {led['dep']:.3f} / {led_r['dep']:.3f}; photo {cnt['photo']} / "
          f"{cnt_r['photo']}, rayleigh {cnt['rayleigh']} / {cnt_r['rayleigh']}, pair "
          f"{cnt['pair']} / {cnt_r['pair']}, annihil {cnt['annihil']} / {cnt_r['annihil']}",
          flush=True)
    assert abs(_closure(led)) < 1e-5
    assert led["dep"] == pytest.approx(led_r["dep"], rel=1e-3)
    frac, nvox = _agreement(d, sg, d_r, sg_r)
    assert nvox > 1000 and frac >= 0.95, frac
    for k, bit in (("photo", 1), ("rayleigh", 2), ("pair", 4), ("moller", 8), ("brem", 16)):
        if physics & bit:
            assert cnt_r[k] > 0
            assert _counts_agree(cnt[k], cnt_r[k]), (k, cnt[k], cnt_r[k])
        else:
            assert cnt[k] == 0
    assert _counts_agree(cnt["annihil"], cnt_r["annihil"]), (cnt["annihil"], cnt_r["annihil"])
    assert _counts_agree(cnt["capped"], cnt_r["capped"]) and cnt["overflow"] == 0
    assert _counts_agree(cnt["real"], cnt_r["real"], rel=2e-3)
    assert _counts_agree(cnt["e_pushed"], cnt_r["e_pushed"], rel=2e-3)


def _pencil(eng, n, e, z0=0.0):
    import torch
    st = eng.Particles(n)
    st.t["x"][:] = 0.1
    st.t["y"][:] = -0.2
    st.t["z"][:] = z0
    st.t["u"][:] = 0.0
    st.t["v"][:] = 0.0
    st.t["w"][:] = 1.0
    st.t["e"][:] = e
    st.t["hid"][:] = torch.arange(n)
    st.t["tag"][:] = 0
    st.t["count"][:] = n
    return st


@pytest.mark.parametrize("e, physics", [(0.04, 7), (0.1, 3), (6.0, 7)],
                         ids=["40keV", "100keV", "6MeV"])
def test_monoenergetic_pencil_matches_oracle(eng, N, orc, wl, e, physics):
    """Monoenergetic photons along +z into a 24 cm water cube through
    transport_batch: at 40 and 100 keV photoelectric absorption and Rayleigh
    scattering are frequent, at 6 MeV pair production and annihilation
    photons (a second photon pass).  Ledger, deposited energy and event
    counts against the oracle on the same streams."""
    import torch
    phs = wl.water_phantom(24, 1.0)
    n = 20000
    print(f"[physics parity] oracle pencil {e} MeV physics={physics}", flush=True)
    _, led_r, cnt_r = orc.transport(phs, 9, np.zeros(n), np.tile([0.1, -0.2, 0.0], (n, 1)),
                                    np.tile([0.0, 0.0, 1.0], (n, 1)), np.full(n, e),
                                    np.arange(n, dtype=np.uint64),
                                    tparams=orc.params(physics=physics))
    print(f"[physics parity] gpu pencil {e} MeV", flush=True)
    ph = eng.Phantom(phs)
    tally = eng.Tally(ph)
    st = _pencil(eng, n, e)
    el = eng.Particles(n * (int(30.0 / 0.2) + 1))
    N.transport_batch(ph.h, st.c, el.c, tally.h, eng.transport_params(physics=physics), 9,
                      eng._stream_ptr())
    torch.cuda.synchronize()
    led, cnt = tally.stats()
    print(f"[physics parity] dep {led['dep']:.4f} / {led_r['dep']:.4f} esc_g {led['esc_g']:.4f} / "
          f"{led_r['esc_g']:.4f}; photo {cnt['photo']} / {cnt_r['photo']}, rayleigh "
          f"{cnt['rayleigh']} / {cnt_r['rayleigh']}, pair {cnt['pair']} / {cnt_r['pair']}, "
          f"annihil {cnt['annihil']} / {cnt_r['annihil']}", flush=True)
    src = n * e
    assert abs(led["esc_g"] + led["esc_e"] + led["dep"] - src) < 1e-5 * src
    assert led["dep"] == pytest.approx(led_r["dep"], rel=3e-3)
    for k in ("photo", "rayleigh", "pair", "annihil", "real", "e_pushed"):
        assert _counts_agree(cnt[k], cnt_r[k]), (k, cnt[k], cnt_r[k])
    if e < 1.0:
        assert cnt["photo"] > 1000 and cnt["rayleigh"] > 100 and cnt["pair"] == 0
    else:
        assert cnt["pair"] > 100 and cnt["annihil"] > 0


@pytest.mark.parametrize("physics", [7, 31], ids=["photons", "all"])
def test_full_physics_graph_equals_eager(eng, wl, physics):
    """The batched runtime with every photon process (annihilation photons in
    a second photon pass per batch), and with the electron hard events too
    (three more generations of passes), replayed from a captured graph, gives
    the eager public-call loop's result."""
    import torch
    W = wl.workload("water60_10x10")
    prm = eng.transport_params(physics=physics)
    model = eng.Model(W.model)
    plan = eng.Plan(model, W.beams, 20000, n_replica=2)
    ph = eng.Phantom(W.phantom)
    t1 = eng.Tally(ph)
    eng.run_plan_eager(plan, ph, t1, prm, 4242, max_batch=1 << 16, band_width=24)
    d1, _ = t1.finalize(plan)
    led1, cnt1 = t1.stats()
    t2 = eng.Tally(ph)
    opts = eng.run_opts(1 << 16, 24, use_graph=True, sort_electrons=True, seed=4242, lane_load=8,
                        pipelines=2)
    for _ in range(2):
        t2.op(eng.N.PSL_TALLY_RESET)
        eng.run_plan(plan, ph, t2, prm, opts)
    d2, _ = t2.finalize(plan)
    torch.cuda.synchronize()
    led2, cnt2 = t2.stats()
    assert abs(_closure(led2)) < 1e-5
    for k in ("photo", "rayleigh", "pair", "annihil", "moller", "brem", "capped", "real",
              "e_pushed", "e_steps", "deposits"):
        assert cnt2[k] == cnt1[k], k
    assert led2["dep"] == pytest.approx(led1["dep"], rel=1e-6)
    hi = d1 > 0.01 * d1.max()
    assert torch.allclose(d2[hi], d1[hi], rtol=1e-4)


def test_pair_needs_cutoff_below_electron_mass(eng, N, wl):
    """Pair production with an electron cut-off above mc^2 is refused: every
    push must cost the photon at least the cut-off for the stack bound.  An
    unknown process bit is refused too."""
    ph = eng.Phantom(wl.water_phantom(8, 1.0))
    tally = eng.Tally(ph)
    st = eng.Particles(64)
    el = eng.Particles(64 * 40)
    st.zero_count()
    with pytest.raises(N.PslError) as e:
        N.transport_batch(ph.h, st.c, el.c, tally.h,
                          eng.transport_params(e_cut_electron=0.6, physics=4), 1,
                          eng._stream_ptr())
    assert e.value.code == N.PSL_EINVAL and "pair" in str(e.value)
    with pytest.raises(N.PslError):
        N.transport_batch(ph.h, st.c, el.c, tally.h, eng.transport_params(physics=32), 1,
                          eng._stream_ptr())


def _electron_pencil(eng, n, e, cap):
    import torch
    st = eng.Particles(cap)
    for f, v in (("x", 0.1), ("y", -0.2), ("z", 0.0), ("u", 0.0), ("v", 0.0), ("w", 1.0), ("e", e)):
        st.t[f][:] = v
    st.t["hid"][:] = torch.arange(cap)
    st.t["tag"][:] = 0
    st.t["count"][:] = n
    st.c.ptype = 1
    return st


@pytest.mark.parametrize("physics", [8, 16, 24, 31], ids=["delta", "brem", "delta_brem", "all"])
def test_electron_pencil_hard_events_match_oracle(eng, N, orc, wl, physics):
    """6 MeV electrons along +z into a 24 cm water cube through
    transport_batch, with Sec. 2.3's cut-offs (0.2 MeV electrons, 0.05 MeV
    photons): Moller delta electrons and bremsstrahlung photons followed for
    three generations.  Ledger, deposited energy and event counts against the
    oracle on the same streams (the GPU reads cross-sections from FP32
    tables, so a decision can tip where a uniform falls within table accuracy
    of its boundary; after that the trajectories are independent samples)."""
    import torch
    phs = wl.water_phantom(24, 1.0)
    n = 20000
    print(f"[electron physics] oracle 6 MeV electron pencil physics={physics}", flush=True)
    _, led_r, cnt_r = orc.transport(phs, 9, np.ones(n), np.tile([0.1, -0.2, 0.0], (n, 1)),
                                    np.tile([0.0, 0.0, 1.0], (n, 1)), np.full(n, 6.0),
                                    np.arange(n, dtype=np.uint64),
                                    tparams=orc.params(e_cut_e=0.2, e_cut_g=0.05, physics=physics))
    print(f"[electron physics] gpu 6 MeV electron pencil physics={physics}", flush=True)
    ph = eng.Phantom(phs)
    tally = eng.Tally(ph)
    # room for the delta electrons of a generation (about one per electron)
    st = _electron_pencil(eng, n, 6.0, 4 * n)
    el = eng.Particles(64)
    N.transport_batch(ph.h, st.c, el.c, tally.h,
                      eng.transport_params(0.2, 0.05, physics=physics), 9, eng._stream_ptr())
    torch.cuda.synchronize()
    led, cnt = tally.stats()
    print(f"[electron physics] dep {led['dep']:.2f} / {led_r['dep']:.2f} esc_g {led['esc_g']:.2f} / "
          f"{led_r['esc_g']:.2f}; moller {cnt['moller']} / {cnt_r['moller']}, brem {cnt['brem']} / "
          f"{cnt_r['brem']}, capped {cnt['capped']} / {cnt_r['capped']}, e_pushed "
          f"{cnt['e_pushed']} / {cnt_r['e_pushed']}", flush=True)
    src = 6.0 * n
    assert abs(led["esc_g"] + led["esc_e"] + led["dep"] - src) < 1e-5 * src
    assert led["dep"] == pytest.approx(led_r["dep"], rel=3e-3)
    assert led["esc_g"] == pytest.approx(led_r["esc_g"], rel=0.05, abs=2.0)
    for k in ("moller", "brem", "capped", "e_pushed", "pair", "annihil", "real"):
        assert _counts_agree(cnt[k], cnt_r[k], rel=0.02), (k, cnt[k], cnt_r[k])
    assert (cnt["moller"] > n // 2) == bool(physics & 8)
    assert (cnt["brem"] > n // 10) == bool(physics & 16)
    assert cnt["overflow"] == 0
