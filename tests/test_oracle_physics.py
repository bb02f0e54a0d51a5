"""Oracle pins for the transport physics (the paper only names the cut-offs,
Sec. 2.3): Klein-Nishina Compton, Bethe stopping power, CSDA range, multiple
scattering sampler."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ME = 0.51099895
RE = 2.8179403262e-13


def _golden(name):
    return [list(map(float, l.split())) for l in open(os.path.join(GOLDEN, name))
            if l.strip() and not l.startswith("#")]


def kn_dsigma_dcos(e, c):
    """Klein-Nishina differential cross-section per unit cos(theta) (cm^2)."""
    k = e / ME
    ratio = 1.0 / (1.0 + k * (1.0 - c))
    return math.pi * RE ** 2 * ratio ** 2 * (ratio + 1.0 / ratio - (1.0 - c * c))


def test_kn_total_golden(orc):
    for e, barn, tol in _golden("kn_total_cross_section.txt"):
        assert orc.kn_sigma(e) / 1e-24 == pytest.approx(barn, rel=tol)


@pytest.mark.parametrize("e", [0.01, 0.05, 0.3, 1.0, 2.5, 6.0])
def test_kn_total_is_integral_of_differential(orc, e):
    val, err = integrate.quad(lambda c: kn_dsigma_dcos(e, c), -1.0, 1.0, epsabs=0,
                              epsrel=1e-12)
    assert orc.kn_sigma(e) == pytest.approx(val, rel=1e-9)


@pytest.mark.parametrize("e", [0.02, 0.4, 2.0, 6.0])
def test_kahn_sampler_histogram(orc, e):
    n = 200000
    cos = orc.kn_sample_cos(e, 99, n)
    assert cos.min() >= -1 - 1e-12 and cos.max() <= 1 + 1e-12
    edges = np.linspace(-1, 1, 41)
    obs = np.histogram(cos, bins=edges)[0]
    tot = orc.kn_sigma(e)
    expv = np.array([integrate.quad(lambda c: kn_dsigma_dcos(e, c), a, b)[0]
                     for a, b in zip(edges[:-1], edges[1:])]) / tot * n
    keep = expv > 20
    chi2 = ((obs[keep] - expv[keep]) ** 2 / expv[keep]).sum()
    dof = keep.sum() - 1
    assert stats.chi2.sf(chi2, dof) > 1e-4
    # Compton edge and mean energy transfer
    k = e / ME
    t = e - e / (1 + k * (1 - cos))
    assert t.max() <= e * 2 * k / (1 + 2 * k) * (1 + 1e-12)
    mean_t = integrate.quad(lambda c: kn_dsigma_dcos(e, c) * (e - e / (1 + k * (1 - c))),
                            -1, 1)[0] / tot
    assert t.mean() == pytest.approx(mean_t, rel=5 * t.std() / mean_t / math.sqrt(n))


def test_bethe_matches_estar(orc):
    for t, s in _golden("estar_water_collision.txt"):
        assert orc.s_col(t) == pytest.approx(s, rel=1e-3)


@pytest.mark.parametrize("t", [0.2000001, 0.25, 0.7, 1.3, 3.0, 6.0])
def test_csda_range_integral_and_inverse(orc, t):
    ref, err = integrate.quad(lambda x: 1.0 / orc.s_col(x), 0.2, t, epsabs=0, epsrel=1e-13,
                              limit=200)
    r = orc.csda_range(t, 0.2)
    assert r == pytest.approx(ref, rel=1e-10, abs=1e-15)
    assert orc.csda_range_inv(r, 0.2) == pytest.approx(t, rel=1e-12)


def test_csda_range_physical_scale(orc):
    # CSDA range of a 1 MeV electron in water is about 0.44 g/cm^2 (ESTAR 0.4367;
    # the Bethe formula without density effect gives a slightly shorter range)
    r = orc.csda_range(1.0, 1e-3) + 0.0
    assert 0.40 < r < 0.45


def test_ms_polar_sampler(orc):
    """A 2D Gaussian in projected angles with width theta0 has a Rayleigh polar
    angle: <theta^2> = 2 theta0^2 and P(theta > x) = exp(-x^2 / (2 theta0^2))."""
    th0 = 0.03
    th = orc.ms_sample(th0, 3, 200000)
    assert np.mean(th ** 2) == pytest.approx(2 * th0 ** 2, rel=0.01)
    assert stats.kstest(th, lambda x: 1 - np.exp(-x ** 2 / (2 * th0 ** 2))).pvalue > 1e-3


def test_highland_zero_and_monotone(orc):
    # structural properties; the constants are pinned against the PDG form below
    assert orc.highland(1.0, 0.0) == 0.0
    assert orc.highland(1.0, 1e-20) == 0.0      # log term clamps the width at 0
    a, b = orc.highland(1.0, 0.01), orc.highland(2.0, 0.01)
    assert a > b > 0


# --- density-effect correction (Sternheimer parametrisation, liquid water) ---

HW_P = 28.816e-6 * math.sqrt(1.0 * 10.0 / 18.0153)   # plasma energy of water, MeV
I_W = 75e-6


def _bg(t):
    tau = t / ME
    return math.sqrt(tau * (tau + 2.0))


@pytest.mark.parametrize("t", [400.0, 1000.0, 5000.0])
def test_density_effect_fermi_limit(orc, t):
    """Above x1 the correction is the high-energy limit
    2 ln(beta gamma) + 2 ln(hbar omega_p / I) - 1, fixed by the electron
    density and I alone (the parametrisation's Cbar must equal
    2 ln(I / hbar omega_p) + 1)."""
    ref = 2.0 * math.log(_bg(t)) + 2.0 * math.log(HW_P / I_W) - 1.0
    assert orc.density_delta(t) == pytest.approx(ref, abs=2e-4)


def test_density_effect_zero_below_x0_and_continuous(orc):
    # x0 = 0.24: beta gamma = 10^0.24
    bg0 = 10 ** 0.24
    t0 = ME * (math.sqrt(1.0 + bg0 * bg0) - 1.0)
    for t in (0.01, 0.1, 0.3, t0 * (1 - 1e-9)):
        assert orc.density_delta(t) == 0.0
        assert orc.s_col(t, density_effect=True) == orc.s_col(t)
    # the middle branch meets the zero branch at x0 (insulator: delta0 = 0)
    assert abs(orc.density_delta(t0 * (1 + 1e-9))) < 5e-4
    # and the Fermi-limit branch at x1 = 2.8004
    bg1 = 10 ** 2.8004
    t1 = ME * (math.sqrt(1.0 + bg1 * bg1) - 1.0)
    assert orc.density_delta(t1 * (1 - 1e-9)) == pytest.approx(orc.density_delta(t1 * (1 + 1e-9)),
                                                              abs=1e-6)
    # delta grows with energy and lowers the stopping power above x0
    ts = np.geomspace(t0 * 1.01, 30.0, 40)
    d = [orc.density_delta(t) for t in ts]
    assert np.all(np.diff(d) > 0)
    for t in ts:
        assert orc.s_col(t, density_effect=True) < orc.s_col(t)


def test_collision_stopping_power_plateau_is_independent_of_i(orc):
    """With the full correction, the Bethe bracket at high energy loses its
    dependence on I: ln(tau^2 (tau+2) / 2) - 2 ln(hbar omega_p / m c^2)
    - 2 ln(beta gamma) + 1 + F-(tau)."""
    t = 1000.0
    tau = t / ME
    g = tau + 1.0
    b2 = 1.0 - 1.0 / g ** 2
    fm = 1.0 - b2 + (tau * tau / 8.0 - (2.0 * tau + 1.0) * math.log(2.0)) / g ** 2
    bracket = (math.log(tau * tau * (tau + 2.0) / 2.0) - 2.0 * math.log(HW_P / ME)
               - 2.0 * math.log(_bg(t)) + 1.0 + fm)
    k = 2.0 * math.pi * RE ** 2 * ME * 6.02214076e23 * 10.0 / 18.0153 / b2
    assert orc.s_col(t, density_effect=True) == pytest.approx(k * bracket, rel=2e-5)


@pytest.mark.parametrize("t", [0.7, 3.0, 6.0])
def test_csda_range_with_density_effect(orc, t):
    ref, err = integrate.quad(lambda x: 1.0 / orc.s_col(x, density_effect=True), 0.2, t,
                              epsabs=0, epsrel=1e-13, limit=200)
    r = orc.csda_range(t, 0.2, density_effect=True)
    assert r == pytest.approx(ref, rel=1e-10)
    assert orc.csda_range_inv(r, 0.2, density_effect=True) == pytest.approx(t, rel=1e-12)
    assert r > orc.csda_range(t, 0.2)


# --- direction rotation, Compton kinematics, Highland width ------------------

def _random_dirs(rng, n):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # directions within 1e-5 of the z axis take the rotation's other branch
    near = np.array([[1e-7, 2e-7, 1.0], [0.0, 0.0, -1.0], [3e-6, -1e-6, -1.0],
                     [0.0, 0.0, 1.0]])
    near /= np.linalg.norm(near, axis=1, keepdims=True)
    return np.vstack([d, near])


def _frame(d):
    """Two unit vectors perpendicular to d and to each other."""
    a = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(d, a)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(d, e1)


def test_rotate_direction_polar_angle_and_norm(orc):
    """The turned direction makes exactly the requested angle with the old one
    and stays a unit vector, on both branches of the rotation."""
    rng = np.random.default_rng(7)
    for d in _random_dirs(rng, 200):
        for c, phi in zip(rng.uniform(-1, 1, 5), rng.uniform(0, 2 * math.pi, 5)):
            n = orc.rotate_direction(d, c, phi)
            assert np.linalg.norm(n) == pytest.approx(1.0, abs=1e-13)
            assert float(n @ d) == pytest.approx(c, abs=1e-12)
    # theta = 0 leaves the direction unchanged, theta = pi reverses it
    for d in _random_dirs(rng, 20):
        assert np.allclose(orc.rotate_direction(d, 1.0, 1.3), d, atol=1e-12)
        assert np.allclose(orc.rotate_direction(d, -1.0, 0.4), -d, atol=1e-12)


def test_rotate_direction_azimuth_is_an_isometry(orc):
    """At fixed theta the azimuth of the new direction about the old one moves
    rigidly with phi (phi -> +-phi + const), so a uniform phi gives a uniform
    azimuth; checked against a frame built independently around d."""
    rng = np.random.default_rng(8)
    for d in _random_dirs(rng, 60):
        e1, e2 = _frame(d)
        c = rng.uniform(-0.95, 0.95)
        phis = rng.uniform(0, 2 * math.pi, 12)
        az = []
        for phi in phis:
            n = orc.rotate_direction(d, c, phi)
            az.append(math.atan2(n @ e2, n @ e1))
        az = np.array(az)
        dphi = np.angle(np.exp(1j * (phis - phis[0])))
        daz = np.angle(np.exp(1j * (az - az[0])))
        same = np.allclose(np.angle(np.exp(1j * (daz - dphi))), 0, atol=1e-9)
        mirror = np.allclose(np.angle(np.exp(1j * (daz + dphi))), 0, atol=1e-9)
        assert same or mirror
    # uniform phi -> uniform azimuth (KS) for one tilted direction
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    e1, e2 = _frame(d)
    az = np.array([math.atan2(n @ e2, n @ e1) for n in
                   (orc.rotate_direction(d, 0.2, p) for p in rng.uniform(0, 2 * math.pi, 4000))])
    assert stats.kstest(az, stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > 1e-3


@pytest.mark.parametrize("e", [0.015, 0.2, 1.0, 5.9])
def test_compton_kinematics_closed_forms(orc, e):
    """Free-electron Compton kinematics: E' = E / (1 + k (1 - cos theta)),
    T = E - E', the electron at cot(theta_e) = (1 + k) tan(theta / 2) on the
    opposite side of the incident direction (azimuth phi + pi), and momentum
    conserved with |p_e| = sqrt(T (T + 2 m c^2))."""
    rng = np.random.default_rng(int(e * 1000))
    k = e / ME
    for d in _random_dirs(rng, 40):
        for _ in range(3):
            cos_t = rng.uniform(-1, 0.999)
            x = 1.0 + k * (1.0 - cos_t)
            phi = rng.uniform(0, 2 * math.pi)
            e1, t, d1, de = orc.compton(e, d, x, phi)
            assert e1 == pytest.approx(e / (1.0 + k * (1.0 - cos_t)), rel=1e-13)
            assert t == pytest.approx(e - e1, rel=1e-12, abs=1e-15)
            assert float(d1 @ d) == pytest.approx(cos_t, abs=1e-12)
            assert np.linalg.norm(de) == pytest.approx(1.0, abs=1e-13)
            th = math.acos(cos_t)
            the = math.acos(max(-1.0, min(1.0, float(de @ d))))
            # cot theta_e = (1 + k) tan(theta / 2)
            assert math.cos(the) * math.cos(th / 2) == pytest.approx(
                (1.0 + k) * math.sin(th / 2) * math.sin(the), abs=1e-10)
            # coplanar with d and d1, on the other side of d
            assert abs(np.linalg.det(np.array([d, d1, de]))) < 1e-10
            if th > 1e-3:
                assert float(np.cross(d, d1) @ np.cross(d, de)) < 0.0
            pe = math.sqrt(t * (t + 2.0 * ME))
            assert np.allclose(e * d, e1 * d1 + pe * de, atol=1e-10 * e)


def _highland_constants():
    return {l.split()[0]: float(l.split()[1]) for l in open(os.path.join(GOLDEN, "highland_pdg.txt"))
            if l.strip() and not l.startswith("#")}


def _tsai_x0(z, a, l_rad, l_rad_p):
    """Radiation length (g/cm^2) from Tsai's formula with the Coulomb correction."""
    alpha = 1.0 / 137.035999084
    az2 = (alpha * z) ** 2
    f = az2 * (1.0 / (1.0 + az2) + 0.20206 - 0.0369 * az2 + 0.0083 * az2 ** 2
               - 0.002 * az2 ** 3)
    inv = 4.0 * alpha * RE ** 2 * 6.02214076e23 / a * (z * z * (l_rad - f) + z * l_rad_p)
    return 1.0 / inv


def test_radiation_length_of_water_from_tsai():
    """X0 of water (the value the Highland width uses) from Tsai's formula for
    hydrogen and oxygen combined by mass fraction, 1/X0 = sum w_i / X0_i."""
    k = _highland_constants()
    x0_h = _tsai_x0(1, 1.008, 5.31, 6.144)
    x0_o = _tsai_x0(8, 15.999, math.log(184.15 * 8 ** (-1 / 3)), math.log(1194.0 * 8 ** (-2 / 3)))
    assert x0_h == pytest.approx(k["X0_hydrogen_g_cm2"], rel=1e-3)
    assert x0_o == pytest.approx(k["X0_oxygen_g_cm2"], rel=1e-3)
    w_h = 2 * 1.008 / (2 * 1.008 + 15.999)
    x0 = 1.0 / (w_h / x0_h + (1 - w_h) / x0_o)
    assert x0 == pytest.approx(k["X0_water_g_cm2"], rel=1e-3)


@pytest.mark.parametrize("t,rho,s", [(0.25, 1.0, 0.05), (1.0, 1.0, 0.125), (3.0, 0.26, 0.4),
                                     (5.5, 1.85, 0.02), (0.6, 1.0, 2.0)])
def test_highland_width_against_pdg(orc, t, rho, s):
    """The step's multiple-scattering width equals the PDG Highland formula with
    beta c p built from the kinetic energy through gamma and beta, and the
    thickness rho s / X0 in radiation lengths of water."""
    k = _highland_constants()
    gamma = 1.0 + t / ME
    beta = math.sqrt(1.0 - 1.0 / gamma ** 2)
    p = gamma * beta * ME                      # MeV/c
    x = rho * s / k["X0_water_g_cm2"]
    ref = k["A_MeV"] / (beta * p) * math.sqrt(x) * (1.0 + k["B"] * math.log(x))
    assert orc.ms_width(t, rho, s) == pytest.approx(ref, rel=1e-12)
    # and the width of a thin step vanishes only where the log term does
    assert orc.ms_width(t, rho, 0.0) == 0.0
