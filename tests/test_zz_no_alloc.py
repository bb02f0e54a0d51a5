"""The allocation-free commissioning solve (commission_nnls_noalloc) against
commission_nnls on the same systems: two calls in a row, the second on a
smaller system, so that the shared scratch array is reused; a system at the
commissioning size; and a system too large for the scratch array."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _system(rng, m, n):
    A = rng.uniform(0, 1, (m, n)) + 0.1 * np.eye(m, n)
    b = A @ rng.uniform(-0.5, 1.5, n) + 0.01 * rng.standard_normal(m)
    return A, b


def _noalloc(N, torch, A, b, x0=None, max_iter=100000):
    m, n = A.shape
    dev = torch.device("cuda")
    a = torch.from_numpy(np.ascontiguousarray(A.T)).to(dev)       # column-major A
    bb = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    x = torch.from_numpy(np.ones(n) if x0 is None else np.array(x0, dtype=np.float64)).to(dev)
    opts = N.psl_nnls_opts(1e-10, 1e-8, 1e-4, 0.5, max_iter)
    rep = N.psl_nnls_report()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    rc = N.commission_nnls_noalloc(a.data_ptr(), m, n, bb.data_ptr(), x.data_ptr(), opts, rep,
                                   C.c_void_p(stream.cuda_stream))
    torch.cuda.synchronize()
    return x.cpu().numpy(), dict(iters=int(rep.iters), f=rep.f, converged=rc == N.PSL_OK)


def test_noalloc_nnls_matches_allocating_solver_twice(eng, N):
    import torch
    rng = np.random.default_rng(7)
    for m, n in ((1000, 300), (300, 80)):
        A, b = _system(rng, m, n)
        x_ref, rep_ref = eng.commission_nnls(A, b)
        x, rep = _noalloc(N, torch, A, b)
        print(f"noalloc nnls {m}x{n}: iters {rep['iters']} vs {rep_ref['iters']}", flush=True)
        assert rep["converged"] and rep_ref["converged"]
        assert rep["f"] == pytest.approx(rep_ref["f"], rel=1e-9)
        assert np.allclose(x, x_ref, atol=2e-5 * np.abs(x_ref).max())
        assert np.array_equal(x == 0, x_ref == 0)


def test_noalloc_nnls_commissioning_size_start_point(eng, N):
    """1656 x 720 (the commissioning system of four fields): zero iterations
    give the projected start point and F there, identically to the
    allocating solver (same kernels, same summation order)."""
    import torch
    rng = np.random.default_rng(8)
    A = rng.uniform(0, 1, (1656, 720))
    b = rng.uniform(0, 1, 1656)
    x0 = rng.uniform(-1, 1, 720)
    x_ref, rep_ref = eng.commission_nnls(A, b, x0=x0, max_iter=0)
    x, rep = _noalloc(N, torch, A, b, x0=x0, max_iter=0)
    assert rep["iters"] == 0 and not rep["converged"]
    assert np.array_equal(x, np.maximum(x0, 0.0))
    assert rep["f"] == rep_ref["f"]


def test_noalloc_nnls_rejects_systems_beyond_the_scratch(N):
    """4000 x 720 needs about 6 MB of scratch: refused before any device work."""
    import torch
    a = torch.zeros(4000 * 720, dtype=torch.float64, device="cuda")
    b = torch.zeros(4000, dtype=torch.float64, device="cuda")
    x = torch.ones(720, dtype=torch.float64, device="cuda")
    opts = N.psl_nnls_opts(1e-10, 1e-8, 1e-4, 0.5, 10)
    rep = N.psl_nnls_report()
    rc = N.lib().commission_nnls_noalloc(a.data_ptr(), 4000, 720, b.data_ptr(), x.data_ptr(),
                                         C.byref(opts), C.byref(rep), None)
    assert rc == N.PSL_EINVAL
    assert b"scratch" in N.lib().psl_last_error()
    assert torch.equal(x, torch.ones_like(x))
