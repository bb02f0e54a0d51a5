"""Oracle pins for the optional photon processes (the paper's engine has the
full photon physics; Sec. 2.3 names only the cut-offs): photoelectric
absorption on oxygen's K shell (Stobbe's hydrogenic cross-section), Rayleigh
scattering with hydrogenic form factors, Bethe-Heitler pair production in
Maximon's expansions, pair energy sharing, positron annihilation, and the
transport with every process switched on."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ME = 0.51099895
RE = 2.8179403262e-13
ALPHA = 7.2973525693e-3
A0 = 0.529177210903e-8
RY = 13.605693122994e-6
HBARC = 1.973269804e-11
SIGMA_T = 8.0 * math.pi / 3.0 * RE ** 2
ALL = 7   # photoelectric | Rayleigh | pair


def _golden(name):
    return [list(map(float, l.split())) for l in open(os.path.join(GOLDEN, name))
            if l.strip() and not l.startswith("#")]


# ---- photoelectric ---------------------------------------------------------
def test_photoeffect_hydrogen_threshold(orc):
    (sigma0, tol), = _golden("photoeffect_hydrogen.txt")
    assert orc.sigma_k_electron(RY * (1.0 + 1e-12), 1.0) == pytest.approx(sigma0, rel=tol)
    assert orc.sigma_k_electron(RY * (1.0 - 1e-9), 1.0) == 0.0


@pytest.mark.parametrize("z", [1.0, 4.55, 7.7])
def test_photoeffect_hydrogenic_scaling(orc, z):
    """A hydrogenic ion of charge z is hydrogen with energies scaled by z^2
    and lengths by 1/z: sigma(E; z) = sigma(E / z^2; 1) / z^2."""
    for e in (2e-3, 1e-2, 0.1, 1.0):
        if e <= z * z * RY:
            continue
        assert orc.sigma_k_electron(e, z) == pytest.approx(
            orc.sigma_k_electron(e / z ** 2, 1.0) / z ** 2, rel=1e-12)


@pytest.mark.parametrize("e", [10.0, 100.0, 1000.0])
def test_photoeffect_high_energy_limit_is_heitler_born(orc, e):
    """Far above the edge Stobbe's result tends to the Born approximation
    (Heitler): per K electron 2 sqrt(2) sigma_T z^5 alpha^4 (mc^2/E)^(7/2),
    with the Coulomb correction 1 - pi nu + O(nu^2), nu = sqrt(I / (E - I))."""
    z = 7.7
    born = 2.0 * math.sqrt(2.0) * SIGMA_T * z ** 5 * ALPHA ** 4 * (ME / e) ** 3.5
    nu = math.sqrt(z * z * RY / (e - z * z * RY))
    ratio = orc.sigma_k_electron(e, z) / born
    assert abs(ratio - (1.0 - math.pi * nu)) < 10.0 * nu * nu


def test_photoelectric_binding_and_attenuation(orc):
    b = orc.photo_binding()
    assert b == pytest.approx(7.7 ** 2 * RY, rel=1e-12)
    # two K electrons per molecule, N_A / 18.0153 molecules per gram
    for e in (0.01, 0.05):
        assert orc.mu_photo(e) == pytest.approx(
            6.02214076e23 / 18.0153 * 2.0 * orc.sigma_k_electron(e, 7.7), rel=1e-12)
    # steeply falling (about E^-3 to E^-3.5 far above the edge)
    slope = math.log(orc.mu_photo(0.1) / orc.mu_photo(0.01)) / math.log(10.0)
    assert -3.6 < slope < -2.9


# ---- Rayleigh ----------------------------------------------------------------
def _radial_ff(q, rho_r2):
    """Form factor of a spherical charge density by quadrature: integral of
    rho(r) r^2 4 pi sin(qr)/(qr) dr, normalised to one electron."""
    norm = integrate.quad(lambda r: rho_r2(r), 0, np.inf, limit=400)[0]
    if q == 0:
        return 1.0
    val = integrate.quad(lambda r: rho_r2(r) * math.sin(q * r) / (q * r), 0, np.inf,
                         limit=400)[0]
    return val / norm


def test_form_factors_are_fourier_transforms_of_hydrogenic_densities(orc):
    """Water's F^2 at t = (q a0)^2 against form factors computed here by
    quadrature from the hydrogenic 1s, 2s, 2p radial densities (a0 = 1)."""
    z1, z2 = 7.70, 4.55
    d1s = lambda z: (lambda r: math.exp(-2 * z * r) * r * r)
    d2s = lambda z: (lambda r: (2 - z * r) ** 2 * math.exp(-z * r) * r * r)
    d2p = lambda z: (lambda r: (z * r) ** 2 * math.exp(-z * r) * r * r)
    for q in (0.0, 0.3, 1.0, 2.5, 7.0, 20.0):
        fh = _radial_ff(q, d1s(1.0))
        fo = (2 * _radial_ff(q, d1s(z1)) + 2 * _radial_ff(q, d2s(z2))
              + 4 * _radial_ff(q, d2p(z2)))
        assert orc.ff2_water(q * q) == pytest.approx(2 * fh * fh + fo * fo, rel=1e-7, abs=1e-12)
    assert orc.ff2_water(0.0) == 66.0


def test_ff_cumulative_is_the_integral(orc):
    for t in (1e-3, 0.5, 3.0, 40.0, 900.0):
        val = integrate.quad(orc.ff2_water, 0.0, t, limit=400, epsrel=1e-12)[0]
        assert orc.ff2_cumulative(t) == pytest.approx(val, rel=1e-9)


def test_rayleigh_limits(orc):
    # low energy: every electron scatters in phase, sigma -> sigma_T F(0)^2
    assert orc.sigma_rayleigh(1e-6) == pytest.approx(SIGMA_T * 66.0, rel=1e-6)
    # high energy: only small angles contribute, sigma E^2 -> pi r_e^2 (hbar c /
    # a0)^2 * 2 * integral_0^inf F^2 dt / 2 (1 + cos^2 -> 2)
    a_inf = orc.ff2_cumulative(1e10)
    lim = math.pi * RE ** 2 * (HBARC / A0) ** 2 * a_inf
    for e in (10.0, 30.0):
        assert orc.sigma_rayleigh(e) * e * e == pytest.approx(lim, rel=2e-3)
    assert orc.mu_rayleigh(0.03) == pytest.approx(
        6.02214076e23 / 18.0153 * orc.sigma_rayleigh(0.03), rel=1e-12)


@pytest.mark.parametrize("e", [0.02, 0.06])
def test_rayleigh_sampler_histogram(orc, e):
    """Sampled cos(theta) against (1 + cos^2) F^2(t(cos)) (chi^2)."""
    n = 60000
    c = orc.rayleigh_sample_cos(e, 17, n)
    x2 = (e * A0 / HBARC) ** 2
    pdf = lambda cc: (1 + cc * cc) * orc.ff2_water(2 * x2 * (1 - cc))
    edges = np.linspace(-1, 1, 41)
    probs = np.array([integrate.quad(pdf, a, b)[0] for a, b in zip(edges[:-1], edges[1:])])
    probs /= probs.sum()
    obs, _ = np.histogram(c, edges)
    exp = probs * n
    keep = exp > 20
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4


# ---- pair production ----------------------------------------------------------
def test_pair_expansions_meet_at_k_4(orc):
    """Maximon's near-threshold and high-energy expansions are independent
    series for the same cross-section; they agree where they meet."""
    lo = orc.sigma_pair_z2(4.0 * ME * (1 - 1e-12))
    hi = orc.sigma_pair_z2(4.0 * ME * (1 + 1e-12))
    assert lo == pytest.approx(hi, rel=3e-4)


def test_pair_threshold_and_high_energy_limit(orc):
    assert orc.sigma_pair_z2(2.0 * ME) == 0.0
    # the cube law at threshold: sigma ~ (2 pi / 3) alpha r_e^2 ((k - 2)/k)^3
    k = 2.0 + 1e-4
    assert orc.sigma_pair_z2(k * ME) == pytest.approx(
        2 * math.pi / 3 * ALPHA * RE ** 2 * ((k - 2) / k) ** 3, rel=1e-3)
    # far above: the unscreened Bethe-Heitler asymptote 28/9 ln 2k - 218/27
    for k in (1e4, 1e5):
        ref = ALPHA * RE ** 2 * (28.0 / 9.0 * math.log(2 * k) - 218.0 / 27.0)
        assert orc.sigma_pair_z2(k * ME) == pytest.approx(ref, rel=1e-5)
    # increasing with energy
    es = np.linspace(1.03, 30.0, 200)
    v = np.array([orc.sigma_pair_z2(x) for x in es])
    assert np.all(np.diff(v) > 0)
    assert orc.mu_pair(6.0) == pytest.approx(
        6.02214076e23 / 18.0153 * 66.0 * orc.sigma_pair_z2(6.0), rel=1e-12)


def test_pair_share_sampler(orc):
    """eps ~ (1 - 4/3 eps (1 - eps)) * 9/7 on [0, 1]: KS test and symmetry."""
    eps = orc.pair_share_sample(23, 100000)
    cdf = lambda x: 9.0 / 7.0 * (x - 2.0 / 3.0 * x * x + 4.0 / 9.0 * x ** 3)
    assert cdf(1.0) == pytest.approx(1.0)
    assert stats.kstest(eps, cdf).pvalue > 1e-4
    assert abs(eps.mean() - 0.5) < 5 * eps.std() / math.sqrt(eps.size)


def test_total_attenuation_parts(orc):
    for e in (0.015, 0.3, 6.0):
        tot, parts = orc.mu_total(e, ALL)
        assert tot == pytest.approx(parts.sum(), rel=1e-15)
        assert parts[0] == pytest.approx(6.02214076e23 * 10 / 18.0153 * orc.kn_sigma(e),
                                         rel=1e-12)
        assert parts[1] == orc.mu_photo(e)
        assert parts[2] == orc.mu_rayleigh(e)
        assert parts[3] == orc.mu_pair(e)
        t0, p0 = orc.mu_total(e, 0)
        assert t0 == parts[0] and p0[1] == p0[2] == p0[3] == 0.0


# ---- transport with every process on -----------------------------------------
def _ledger_residual(led):
    out = led["jaw"] + led["missed"] + led["invalid"] + led["esc_g"] + led["esc_e"] + led["dep"]
    return (led["src"] - out) / led["src"]


@pytest.mark.parametrize("e", [0.03, 6.0])
def test_ledger_closes_with_every_process(orc, wl, e):
    """Monoenergetic pencil beams into water: energy is conserved exactly
    with photoelectric absorption, Rayleigh scattering, pair production and
    annihilation photons followed as histories of their own."""
    ph = wl.water_phantom(24, 1.0)
    n = 4000
    pos = np.tile([0.1, -0.2, 0.0], (n, 1))
    dirs = np.tile([0.0, 0.0, 1.0], (n, 1))
    tp = orc.params(physics=ALL)
    edep, led, cnt = orc.transport(ph, 5, np.zeros(n), pos, dirs, np.full(n, e),
                                   np.arange(n, dtype=np.uint64), tparams=tp)
    assert abs(_ledger_residual(led)) < 1e-12
    assert led["dep"] == pytest.approx(edep.sum(), rel=1e-12)
    if e < 0.1:
        assert cnt["photo"] > 0 and cnt["rayleigh"] > 0 and cnt["pair"] == 0
    else:
        assert cnt["pair"] > 0
        # each positron that stops inside annihilates once
        assert 0 < cnt["annihil"] <= cnt["pair"]


def test_uncollided_transmission_with_every_process(orc, wl):
    """exp(-sum mu l) with mu the sum of all four processes."""
    slabs = [(10, 1.0), (8, 0.26), (4, 1.85), (6, 1.0)]
    ph = wl.slab_phantom(5, 1.0, slabs, 0.5)
    n = 200000
    for e in (0.04, 3.0):
        pos = np.tile([0.01, -0.02, 0.0], (n, 1))
        dirs = np.tile([0.0, 0.0, 1.0], (n, 1))
        _, led, cnt = orc.transport(ph, 3, np.zeros(n), pos, dirs, np.full(n, e),
                                    np.arange(n, dtype=np.uint64), tparams=orc.params(physics=ALL))
        mu = orc.mu_total(e, ALL)[0]
        p = math.exp(-sum(mu * rho * k * 0.5 for k, rho in slabs))
        frac = cnt["esc_uncollided"] / n
        assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / n)


def test_process_frequencies_follow_the_attenuations(orc, wl):
    """In a water sheet 0.05 cm thick a 40 keV photon interacts at most once
    in practice (1.3 % interact, a second interaction is 1e-4 likely): the
    real collisions split into Compton, photoelectric and Rayleigh in
    proportion to the attenuations (chi^2)."""
    e = 0.04
    tot, parts = orc.mu_total(e, ALL)
    ph = wl.slab_phantom(4, 2.0, [(1, 1.0)], 0.05)
    n = 400000
    pos = np.tile([0.0, 0.0, 0.0], (n, 1))
    dirs = np.tile([0.0, 0.0, 1.0], (n, 1))
    _, led, cnt = orc.transport(ph, 41, np.zeros(n), pos, dirs, np.full(n, e),
                                np.arange(n, dtype=np.uint64), tparams=orc.params(physics=ALL))
    assert abs(_ledger_residual(led)) < 1e-12
    assert cnt["pair"] == 0
    obs = np.array([cnt["real"] - cnt["photo"] - cnt["rayleigh"], cnt["photo"], cnt["rayleigh"]])
    exp = parts[:3] / parts[:3].sum() * obs.sum()
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, 2) > 1e-4, (obs, exp)
    assert obs.sum() > 3000
