"""Commissioning path on the GPU (Sec. 2.2.2-2.2.4): all fields and all basis
doses of a stratified plan in one run through the index-map tally, compared
with the oracle; column sums reproduce the open-field dose; the NNLS fit of
the GPU-built matrix recovers the seeded weights."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HPB = 400      # histories per (field, basis); the full workload uses 1e6


@pytest.fixture(scope="module")
def commission(eng, orc, wl):
    import torch
    W = wl.workload("commission60")
    imap, n_rows = W.extra["index_map"], W.extra["n_rows"]
    bmap = W.extra["basis_map"]
    n_cols = len(W.beams) * 720
    model = eng.Model(W.model)
    plan = eng.Plan(model, W.beams, 0, n_replica=2, basis_map=bmap, hist_per_basis=HPB)
    ph = eng.Phantom(W.phantom)
    tally = eng.Tally(ph, index_map=imap, n_rows=n_rows, n_cols=n_cols)
    prm = eng.transport_params()
    print(f"[commission] gpu run, {plan.n_hist} histories per replica", flush=True)
    eng.run_plan(plan, ph, tally, prm, eng.run_opts(262144, 24, use_graph=True, seed=31))
    A, sA = tally.finalize(plan)
    torch.cuda.synchronize()
    led, cnt = tally.stats()
    ref_w, _ = orc.psl_build(W.model)
    op = orc.plan_build(W.model, ref_w, W.beams, 0, basis_map=bmap, hist_per_basis=HPB)
    print("[commission] oracle run", flush=True)
    s, s2, led_ref, cnt_ref = orc.run(W.model, op, W.beams, W.phantom, 31, 2, index_map=imap,
                                      n_rows=n_rows, n_cols=n_cols)
    return dict(W=W, plan=plan, A=A.cpu().numpy(), sA=sA.cpu().numpy(), led=led, cnt=cnt,
                s=s.reshape(n_rows, n_cols), s2=s2.reshape(n_rows, n_cols), led_ref=led_ref,
                op=op, n_rows=n_rows, n_cols=n_cols, imap=imap)


def test_commission_tally_matches_oracle(commission):
    c = commission
    assert c["plan"].n_hist == c["op"].n_hist
    assert c["led"]["dep"] == pytest.approx(c["led_ref"]["dep"], rel=1e-3)
    # energy per cell, summed over the two replicas (shared streams)
    col_w = c["plan"].col_weight()
    rho_v = 1.0
    vol = 0.5 ** 3
    k = 1.602176634e-10 * col_w[None, :] / (rho_v * vol)
    a_ref = k * c["s"] / 2.0
    tot, tot_ref = c["A"].sum(), a_ref.sum()
    assert tot == pytest.approx(tot_ref, rel=2e-3)
    hi = a_ref > 0.1 * a_ref.max()
    assert hi.sum() > 100
    rel = np.abs(c["A"][hi] - a_ref[hi]) / a_ref[hi]
    assert np.median(rel) < 1e-3


def test_columns_sum_to_open_field_dose(eng, wl):
    """Sum over the basis columns of one field (x = 1) equals the Eq. (3)
    open-field dose on the same voxels within the statistical error (GPU
    only, 2e4 histories per basis so that the per-PSL allocation of the
    stratified counts is fine enough)."""
    import torch
    W = wl.workload("commission60")
    imap, n_rows = W.extra["index_map"], W.extra["n_rows"]
    bmap = W.extra["basis_map"]
    beam = W.beams[2]                                   # 10 x 10 field
    model = eng.Model(W.model)
    ph = eng.Phantom(W.phantom)
    prm = eng.transport_params()
    plan_c = eng.Plan(model, [beam], 0, n_replica=4, basis_map=bmap, hist_per_basis=20000)
    tally_c = eng.Tally(ph, index_map=imap, n_rows=n_rows, n_cols=720)
    eng.run_plan(plan_c, ph, tally_c, prm, eng.run_opts(1 << 20, 24, seed=41))
    A, sA = tally_c.finalize(plan_c)
    plan = eng.Plan(model, [beam], 4000000, n_replica=4)
    tally = eng.Tally(ph)
    eng.run_plan(plan, ph, tally, prm, eng.run_opts(1 << 20, 24, seed=5))
    d, s = tally.finalize(plan)
    torch.cuda.synchronize()
    A, sA = A.cpu().numpy(), sA.cpu().numpy()
    d = d.cpu().numpy().ravel()
    s = s.cpu().numpy().ravel()
    sel = np.flatnonzero(imap.ravel())
    rows = imap.ravel()[sel] - 1
    a_field = A.sum(axis=1)
    sa_field = np.sqrt((sA ** 2).sum(axis=1))
    open_d = np.zeros(n_rows)
    open_s = np.zeros(n_rows)
    open_d[rows] = d[sel]
    open_s[rows] = s[sel]
    hi = open_d > 0.2 * open_d.max()
    z = (a_field[hi] - open_d[hi]) / np.sqrt(sa_field[hi] ** 2 + open_s[hi] ** 2)
    assert hi.sum() > 50
    assert np.mean(np.abs(z) < 3) > 0.95
    assert abs(np.mean(z)) < 0.5
    # integral over the selected voxels within 0.5 %
    assert a_field[hi].sum() == pytest.approx(open_d[hi].sum(), rel=5e-3)


def test_nnls_fit_of_gpu_matrix(eng, orc, wl, commission):
    """Noise-free target b = A x_true from the GPU-built basis matrix: both
    gradient-projection solvers (GPU and oracle) reduce the residual to
    1e-3 of |b| within the same iteration budget (the matrix is too
    ill-conditioned for full convergence, so the iterates are not compared)."""
    c = commission
    A = c["A"]
    used = A.max(axis=0) > 0
    A = A[:, used]
    x_true, b = wl.commissioning_target(A, 11, noise_rel=0.0)
    scale = b.max()
    x, rep = eng.commission_nnls(A / scale, b / scale, max_iter=20000)
    xo, repo = orc.nnls_gp(A / scale, b / scale, max_iter=20000)
    for xx in (x, xo):
        assert np.all(xx >= 0)
        assert np.linalg.norm(A @ xx - b) < 1e-3 * np.linalg.norm(b)
    assert rep["f"] < 1e-6 * np.sum((b / scale) ** 2)
