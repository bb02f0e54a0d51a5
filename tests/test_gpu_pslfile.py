"""The particle-file source path: sample_batch(PSL_SAMPLE_PLANE) records,
stored to disk and read back, then psl_transform_batch, give bit for bit the
stack that the fused sampler writes (sample_batch with PSL_SAMPLE_DENSE), and
the source ledger splits between the two calls without loss; a dose
calculated from the files equals the on-the-fly dose to FP32 atomic-add
rounding with identical event counters."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def test_plane_records_then_transform_equal_fused(eng, N, wl, tmp_path):
    import torch
    from paper_1503_01725_amd import pslfile as pf
    W = wl.workload("hetero256_5beam")
    model = eng.Model(W.model)
    plan = eng.Plan(model, W.beams, 200000, n_replica=2)
    ph = eng.Phantom(W.phantom)
    t_fused, t_plane = eng.Tally(ph), eng.Tally(ph)
    nb = plan.set_batching(1 << 30, 24)   # one batch per (beam, sub-source)
    seed, rep = 0xF11E, 1
    beams_seen = set()
    for i in range(nb):
        b = plan.batch(i)
        print(f"[pslfile parity] batch {i} stype {b.stype} h0 {b.h0} n {b.n}", flush=True)
        fused = eng.Particles(b.n)
        N.sample_batch(plan.h, ph.h, rep, b.h0, b.n, seed, fused.c, N.PSL_SAMPLE_DENSE,
                       t_fused.h, eng._stream_ptr())
        plane = eng.Particles(b.n)
        N.sample_batch(plan.h, ph.h, rep, b.h0, b.n, seed, plane.c, N.PSL_SAMPLE_PLANE,
                       t_plane.h, eng._stream_ptr())
        torch.cuda.synchronize()
        pr = plane.host(b.n)
        assert np.all(pr["z"] == 0.0)
        assert set(np.unique(pr["status"])) <= {0, 3}
        beams_seen |= set(np.unique(pr["sub"][pr["status"] == 0]).tolist())
        rec = {f: pr[f] for f in pf.FLOAT_FIELDS}
        rec["hid"] = pr["hid"]
        rec["tag"] = (pr["tag"].astype(np.uint32) | (pr["sub"].astype(np.uint32) << 16)
                      | (pr["status"].astype(np.uint32) << 24))
        path = str(tmp_path / f"b{i}.psl")
        size = pf.write_records(path, rec, 1 if b.stype == 2 else 0)
        src = pf.FileSource(size)
        n, ptype, got = src.read(path)
        assert (n, got) == (b.n, size) and ptype == (1 if b.stype == 2 else 0)
        src.copy(got)
        out = eng.Particles(b.n)
        N.psl_transform_batch(plan.h, ph.h, src.plane_stack(n, ptype), n, out.c, t_plane.h,
                              eng._stream_ptr())
        torch.cuda.synchronize()
        assert out.count() == b.n
        fr, tr = fused.host(b.n), out.host(b.n)
        for f in ("x", "y", "z", "u", "v", "w", "e"):
            assert np.array_equal(_bits(tr[f]), _bits(fr[f])), f
        for f in ("hid", "tag", "sub", "status"):
            assert np.array_equal(tr[f], fr[f]), f
    assert beams_seen == set(range(len(W.beams)))
    lf, cf = t_fused.stats()
    lp, cp = t_plane.stats()
    for k in ("src", "jaw", "missed", "invalid"):
        assert lp[k] == pytest.approx(lf[k], rel=1e-12, abs=1e-9), k
    for k in ("hist", "entered"):
        assert int(cp[k]) == int(cf[k]), k


def test_dose_from_files_matches_on_the_fly(eng, N, wl, tmp_path):
    from paper_1503_01725_amd import pslfile as pf
    import os
    W = wl.workload("water60_10x10")
    model = eng.Model(W.model)
    plan = eng.Plan(model, W.beams, 300000, n_replica=1)
    ph = eng.Phantom(W.phantom)
    prm = eng.transport_params()
    mb, bw = 65536, 4
    gen = eng.Tally(ph)
    paths, total = pf.generate(plan, ph, gen, W.seed, str(tmp_path), mb, bw, log=lambda m: None)
    assert total == sum(os.path.getsize(p) for p in paths)
    t_o, t_f = eng.Tally(ph), eng.Tally(ph)
    pf.run_on_the_fly(plan, ph, t_o, prm, W.seed, mb, bw)
    src = pf.FileSource(max(os.path.getsize(p) for p in paths))
    tf = pf.run_from_files(paths, plan, ph, t_f, prm, W.seed, mb, src)
    assert tf["rd"] > 0 and tf["sim"] > 0
    d_o, _ = t_o.finalize(plan)
    d_f, _ = t_f.finalize(plan)
    d_o, d_f = d_o.cpu().numpy(), d_f.cpu().numpy()
    assert np.abs(d_o - d_f).max() <= 1e-5 * np.abs(d_o).max()
    _, co = t_o.stats()
    _, cf = t_f.stats()
    for k in ("entered", "wc_steps", "real", "e_pushed", "e_local", "e_steps", "deposits",
              "kahn_trials", "e_boundary"):
        assert int(co[k]) == int(cf[k]), k
