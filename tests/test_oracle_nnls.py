"""Oracle pins for the commissioning solve (Sec. 2.2.3 Eq. 8, Sec. 2.2.4):
gradient projection with Armijo's rule against scipy's Lawson-Hanson NNLS, the
KKT conditions, and exact recovery from noise-free data."""
import numpy as np
import pytest
from scipy.optimize import nnls


def _kkt(A, b, x, tol):
    g = 2 * A.T @ (A @ x - b)
    scale = np.abs(g).max() + np.abs(2 * A.T @ b).max()
    assert np.all(x >= 0)
    assert np.all(g[x == 0] >= -tol * scale)
    assert np.all(np.abs(g[x > 0]) <= tol * scale)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gp_matches_lawson_hanson(orc, seed):
    rng = np.random.default_rng(seed)
    m, n = 120, 40
    A = rng.uniform(0, 1, (m, n)) + 0.1 * np.eye(m, n)
    x_true = rng.uniform(-0.5, 1.5, n)          # some components want to be < 0
    b = A @ x_true + 0.01 * rng.standard_normal(m)
    x, rep = orc.nnls_gp(A, b)
    xr, rr = nnls(A, b)
    f_ref = rr ** 2
    assert rep["converged"]
    assert rep["f"] == pytest.approx(f_ref, rel=1e-8)
    assert np.allclose(x, xr, atol=2e-5 * np.abs(xr).max())
    assert np.array_equal(x == 0, xr == 0)       # same active set
    assert np.count_nonzero(xr == 0) > 0
    _kkt(A, b, x, 1e-7)


def test_gp_recovers_noise_free_target(orc):
    rng = np.random.default_rng(7)
    m, n = 300, 60
    A = np.abs(rng.standard_normal((m, n))) + 0.05
    x_true = rng.uniform(0.8, 1.2, n)
    b = A @ x_true
    x, rep = orc.nnls_gp(A, b, delta=1e-14, pg_tol=1e-12)
    assert np.allclose(x, x_true, rtol=1e-6)


def test_gp_reports_nonconvergence(orc):
    rng = np.random.default_rng(3)
    A = rng.uniform(0, 1, (50, 30))
    b = rng.uniform(0, 1, 50)
    x, rep = orc.nnls_gp(A, b, max_iter=3)
    assert rep["iters"] == 3 and not rep["converged"]
    assert np.all(x >= 0)
