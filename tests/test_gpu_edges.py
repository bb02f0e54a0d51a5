"""Edge cases of the dose path on the GPU: empty particle stacks, plans of one
or a few histories per replica (single-history batches, more pipelines asked
for than batches, ragged batch ends) against the oracle, and the launch and
size limits the library refuses before any device work."""
import pytest

pytestmark = pytest.mark.gpu

LEDGER_OUT = ("jaw", "missed", "invalid", "esc_g", "esc_e", "dep")


def test_empty_stacks_deposit_nothing(eng, N, wl):
    """A photon stack and an electron stack that hold no entries: both
    transport calls return, nothing is deposited or counted, and the one fold
    is the only event."""
    import torch
    W = wl.workload("water60_10x10")
    ph = eng.Phantom(W.phantom)
    tally = eng.Tally(ph)
    prm = eng.transport_params()
    photons, electrons = eng.Particles(256), eng.Particles(1024)
    photons.zero_count()
    electrons.zero_count()
    tally.op(N.PSL_TALLY_RESET)
    print("[edges] empty photon stack", flush=True)
    N.transport_batch(ph.h, photons.c, electrons.c, tally.h, prm, 3, eng._stream_ptr())
    electrons.c.ptype = 1
    print("[edges] empty electron stack", flush=True)
    N.transport_batch(ph.h, electrons.c, electrons.c, tally.h, prm, 3, eng._stream_ptr())
    tally.op(N.PSL_TALLY_FOLD)
    torch.cuda.synchronize()
    led, cnt = tally.stats()
    assert electrons.count() == 0
    assert all(v == 0.0 for v in led.values()), led
    assert cnt["folds"] == 1
    assert all(v == 0 for k, v in cnt.items() if k != "folds"), cnt


@pytest.mark.parametrize("n_hist", [1, 7, 97])
def test_tiny_plans_match_oracle(eng, N, orc, wl, n_hist):
    """One, seven and 97 histories per replica, three replicas, through the
    batched runtime as one captured graph with two pipelines asked for (a
    one-history plan has a single batch, so one pipeline runs): the history
    count, the folds and the source ledger (sampled energy, jaw-rejected and
    missed) equal the oracle's on the same streams, and the energy ledger
    closes."""
    import torch
    W = wl.workload("water60_10x10")
    model = eng.Model(W.model)
    plan = eng.Plan(model, W.beams, n_hist, n_replica=3)
    ph = eng.Phantom(W.phantom)
    tally = eng.Tally(ph)
    prm = eng.transport_params()
    print(f"[edges] {n_hist} histories x 3 replicas, graph, two pipelines asked", flush=True)
    eng.run_plan(plan, ph, tally, prm, eng.run_opts(4096, 24, use_graph=True, seed=11,
                                                    sort_electrons=False, lane_load=32,
                                                    pipelines=2))
    torch.cuda.synchronize()
    led, cnt = tally.stats()
    ref_w, _ = orc.psl_build(W.model)
    op = orc.plan_build(W.model, ref_w, W.beams, n_hist)
    _, _, led_ref, cnt_ref = orc.run(W.model, op, W.beams, W.phantom, 11, 3)
    assert cnt["hist"] == cnt_ref["hist"] == 3 * n_hist
    assert cnt["folds"] == 3
    assert cnt["entered"] == cnt_ref["entered"]
    for k in ("src", "jaw", "missed"):
        assert led[k] == pytest.approx(led_ref[k], rel=1e-6, abs=1e-9), k
    assert abs(led["src"] - sum(led[k] for k in LEDGER_OUT)) <= 1e-6 * led["src"]


def test_run_limits_are_refused(eng, N, wl):
    """Launch options outside the runtime's limits fail with an error before
    any stack is allocated: batches below 64 histories, band width 0, more
    than two pipelines, more than 4096 histories per lane, and a batch whose
    electron stack would pass 2^32 entries."""
    W = wl.workload("water60_10x10")
    model = eng.Model(W.model)
    plan = eng.Plan(model, W.beams, 1000, n_replica=1)
    ph = eng.Phantom(W.phantom)
    tally = eng.Tally(ph)
    prm = eng.transport_params()
    bad = [dict(max_batch=32, band_width=24), dict(max_batch=4096, band_width=0),
           dict(max_batch=4096, band_width=24, pipelines=3),
           dict(max_batch=4096, band_width=24, lane_load=5000),
           dict(max_batch=(1 << 30) + 64, band_width=24)]
    for kw in bad:
        print(f"[edges] refused options {kw}", flush=True)
        with pytest.raises(N.PslError):
            eng.run_plan(plan, ph, tally, prm, eng.run_opts(use_graph=False, seed=1, **kw))
    led, cnt = tally.stats()
    assert cnt["hist"] == 0


def test_size_limits_are_refused(eng, N):
    """Phantoms of 2^31 voxels or more, empty phantom axes, U-Net volumes that
    four levels cannot halve (not multiples of 8) or that exceed its index
    range, and unsupported widths are refused with an error before any device
    memory is touched or allocated."""
    import ctypes as C
    import torch
    buf = torch.zeros(64, dtype=torch.float32, device="cuda")
    for nx, ny, nz in ((2048, 2048, 512), (0, 4, 4)):
        print(f"[edges] refused phantom {nx} x {ny} x {nz}", flush=True)
        with pytest.raises(N.PslError):
            N.psl_phantom_create(buf.data_ptr(), nx, ny, nz, (0.1, 0.1, 0.1), (0.0, 0.0, 0.0))
    out = C.c_void_p()
    for c, d, h, w in ((8, 12, 16, 16), (8, 16, 16, 4), (8, 1024, 1024, 512), (24, 16, 16, 16)):
        print(f"[edges] refused U-Net width {c} at {d} x {h} x {w}", flush=True)
        assert N.lib().psl_unet_create(c, d, h, w, C.byref(out)) == N.PSL_EINVAL
    assert not out.value
