// Host-built physics tables for the transport kernels (FP64 on the host,
// stored as FP32 for the device):
//   * n_e * sigma_KN(E): free-electron Klein-Nishina total cross-section times
//     the electron density of water at unit mass density (1/cm), on a log-E grid;
//   * R(T): CSDA range above the electron cut-off, integral of 1/S_col with the
//     Bethe collision stopping power of water (ICRU 37 form, I = 75 eV), with
//     or without Sternheimer's density-effect correction, on a log-T grid;
//   * T(R): its inverse, on a grid uniform in ln(R + R_off).
#include <cmath>

#include "common.hpp"

namespace psl {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMe = 0.51099895000;          // MeV
constexpr double kRe = 2.8179403262e-13;       // cm
constexpr double kNa = 6.02214076e23;          // 1/mol
constexpr double kZoverA = 10.0 / 18.0153;     // water, mol/g
constexpr double kIwater = 75.0e-6;            // MeV
constexpr double kEmin = 1.0e-3, kEmax = 30.0; // photon table range, MeV
constexpr double kTmax = 30.0;                 // electron table top, MeV
constexpr double kROff = 1.0e-4;               // g/cm^2, offset of the inverse grid
// Density-effect parameters of liquid water (Sternheimer, Berger and Seltzer
// 1984): delta = 2 ln10 x - Cbar + a (x1 - x)^m on [x0, x1), 2 ln10 x - Cbar
// above x1 and 0 below x0, where x = log10(p / m c).
constexpr double kCbar = 3.5017, kX0 = 0.2400, kX1 = 2.8004, kDa = 0.09116, kDm = 3.4773;

double klein_nishina(double e) {
    const double k = e / kMe;
    const double a = 1.0 + 2.0 * k;
    const double la = std::log(a);
    const double t1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - la / k);
    const double t2 = la / (2.0 * k);
    const double t3 = (1.0 + 3.0 * k) / (a * a);
    return 2.0 * kPi * kRe * kRe * (t1 + t2 - t3);
}

double density_delta(double t) {
    const double tau = t / kMe;
    const double x = 0.5 * std::log10(tau * (tau + 2.0));
    if (x < kX0) return 0.0;
    const double lin = 2.0 * std::log(10.0) * x - kCbar;
    return x < kX1 ? lin + kDa * std::pow(kX1 - x, kDm) : lin;
}

// kinetic energy at log10(p / m c) = x
double t_at_x(double x) {
    const double p = std::pow(10.0, x);
    return kMe * (std::sqrt(1.0 + p * p) - 1.0);
}

double bethe(double t, bool dens) {
    const double tau = t / kMe;
    const double gamma = 1.0 + tau;
    const double b2 = 1.0 - 1.0 / (gamma * gamma);
    const double ir = kIwater / kMe;
    const double fm = 1.0 - b2 + (0.125 * tau * tau - (2.0 * tau + 1.0) * std::log(2.0)) / (gamma * gamma);
    const double lg = std::log(tau * tau * (tau + 2.0) / (2.0 * ir * ir));
    const double d = dens ? density_delta(t) : 0.0;
    return 2.0 * kPi * kRe * kRe * kMe * kNa * kZoverA * (lg + fm - d) / b2;
}

// Simpson integral of 1/S over [a, b] with m (even) panels; with the density
// effect the integrand has a kink where delta leaves zero (x0) and another at
// x1, and an interval across one is split there.
double inv_s_integral(double a, double b, int m, bool dens) {
    if (dens) {
        for (double k : {t_at_x(kX0), t_at_x(kX1)})
            if (a < k && k < b) return inv_s_integral(a, k, m, dens) + inv_s_integral(k, b, m, dens);
    }
    const double h = (b - a) / m;
    double s = 1.0 / bethe(a, dens) + 1.0 / bethe(b, dens);
    for (int i = 1; i < m; ++i) s += (i % 2 ? 4.0 : 2.0) / bethe(a + i * h, dens);
    return s * h / 3.0;
}

}  // namespace

void ensure_physics(psl_phantom* ph, const psl_transport_params* p) {
    PSL_CHECK(p->density_effect == 0 || p->density_effect == 1, "density_effect must be 0 or 1");
    const bool dens = p->density_effect == 1;
    if (ph->t_cut_tab == p->e_cut_electron && ph->dens_tab == p->density_effect && ph->tabs.p) return;
    const double tcut = p->e_cut_electron;
    PSL_CHECK(tcut > 2.0e-3 && tcut < 10.0, "e_cut_electron must be in (0.002, 10) MeV");
    // A photon pays at least the cut-off for every electron it sets in
    // motion, and the electron's random sub-stream id (1 + its push index)
    // has 8 bits in the particle tag: photons up to the top of the tables
    // must not push more than 255 electrons.
    PSL_CHECK(std::floor(kEmax / tcut) <= 255.0,
              "e_cut_electron must be at least %.4f MeV (at most 255 electrons per photon of "
              "up to %.0f MeV)", kEmax / 255.0, kEmax);

    std::vector<float> host(size_t(KN_TAB_N) + RNG_TAB_N + INV_TAB_N);
    float* kn = host.data();
    float* rng = kn + KN_TAB_N;
    float* inv = rng + RNG_TAB_N;

    const double ne = kNa * kZoverA;
    const double le0 = std::log(kEmin), dle = (std::log(kEmax) - le0) / (KN_TAB_N - 1);
    for (int i = 0; i < KN_TAB_N; ++i) kn[i] = float(ne * klein_nishina(std::exp(le0 + i * dle)));

    // fine FP64 range table on a log grid, 16 Simpson panels per interval
    const int fine = 16 * (RNG_TAB_N - 1) + 1;
    const double lt0 = std::log(tcut), dlf = (std::log(kTmax) - lt0) / (fine - 1);
    std::vector<double> tf(fine), rf(fine);
    tf[0] = tcut;
    rf[0] = 0.0;
    for (int i = 1; i < fine; ++i) {
        tf[i] = std::exp(lt0 + i * dlf);
        rf[i] = rf[i - 1] + inv_s_integral(tf[i - 1], tf[i], 8, dens);
    }
    for (int i = 0; i < RNG_TAB_N; ++i) rng[i] = float(rf[size_t(i) * 16]);
    // inverse on u = ln(R + R_off): monotone interpolation in the fine table,
    // refined by Newton steps on the exact integral
    const double r_max = rf[fine - 1];
    const double u0 = std::log(kROff), du = (std::log(r_max + kROff) - u0) / (INV_TAB_N - 1);
    size_t k = 0;
    for (int i = 0; i < INV_TAB_N; ++i) {
        double r = std::exp(u0 + i * du) - kROff;
        if (i == 0) r = 0.0;
        if (r > r_max) r = r_max;
        while (k + 1 < size_t(fine) - 1 && rf[k + 1] < r) ++k;
        double t = tf[k] + (tf[k + 1] - tf[k]) * (r - rf[k]) / (rf[k + 1] - rf[k]);
        for (int it = 0; it < 4; ++it) {
            const double rt = rf[k] + inv_s_integral(tf[k], t, 8, dens);
            t -= (rt - r) * bethe(t, dens);
        }
        inv[i] = float(t);
    }
    ph->tabs.upload(host);
    PhysicsDev& d = ph->phys;
    d.kn_lne0 = float(le0);
    d.kn_inv_dlne = float(1.0 / dle);
    d.rng_lnt0 = float(lt0);
    d.rng_inv_dlnt = float(1.0 / (dlf * 16));
    d.inv_u0 = float(u0);
    d.inv_inv_du = float(1.0 / du);
    d.r_off = float(kROff);
    d.r_tab_max = float(r_max);
    d.t_cut = float(tcut);
    d.t_max = float(kTmax);
    d.kn = ph->tabs.as<float>();
    d.rng = d.kn + KN_TAB_N;
    d.inv = d.rng + RNG_TAB_N;
    ph->t_cut_tab = p->e_cut_electron;
    ph->dens_tab = p->density_effect;
    ++ph->tab_gen;
}

}  // namespace psl
