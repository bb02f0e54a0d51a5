// Host-built physics tables for the transport kernels (FP64 on the host,
// stored as FP32 for the device):
//   * n_e * sigma_KN(E): free-electron Klein-Nishina total cross-section times
//     the electron density of water at unit mass density (1/cm), on a log-E grid;
//   * R(T): CSDA range above the electron cut-off, integral of 1/S_col with the
//     Bethe collision stopping power of water (ICRU 37 form, I = 75 eV), with
//     or without Sternheimer's density-effect correction, on a log-T grid;
//   * T(R): its inverse, on a grid uniform in ln(R + R_off);
//   * with optional photon processes: the cumulative attenuations (Compton,
//     + photoelectric, + Rayleigh, + pair) per unit density on the log-E
//     grid, and the cumulative integral of the molecule's squared form factor
//     for sampling the Rayleigh angle;
//   * with optional electron hard events (Moller delta rays, bremsstrahlung):
//     R(T) of the continuous loss left below the cut-offs (the collision
//     stopping power restricted to transfers below the electron cut-off, the
//     radiative loss to photons below the photon cut-off) and the hard-event
//     cross-sections per unit density on the range table's grid.
#include <algorithm>
#include <cmath>
#include <vector>

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

// ---- optional electron hard events (water) ------------------------------------
constexpr double kAlphaFs = 7.2973525693e-3;
constexpr double kZZ1Water = 76.0;              // sum of Z (Z + 1) over H2O

// Collision stopping power restricted to energy transfers below tc (ICRU 37,
// the Rohrlich-Carlson F-(tau, Delta), Delta = tc / mc^2 at most tau / 2).
double bethe_restricted(double t, double tc, bool dens) {
    const double tau = t / kMe, gamma = 1.0 + tau, b2 = 1.0 - 1.0 / (gamma * gamma);
    const double ir = kIwater / kMe;
    const double dl = std::min(tc / kMe, 0.5 * tau);
    const double fm = -1.0 - b2 + std::log((tau - dl) * dl) + tau / (tau - dl) +
                      (0.5 * dl * dl + (2.0 * tau + 1.0) * std::log(1.0 - dl / tau)) / (gamma * gamma);
    const double d = dens ? density_delta(t) : 0.0;
    return 2.0 * kPi * kRe * kRe * kMe * kNa * kZoverA *
           (std::log(2.0 * (tau + 2.0) / (ir * ir)) + fm - d) / b2;
}

// Moller collisions transferring [tc, t/2] per unit density (cm^2/g), the
// closed form of the Moller cross-section's integral.
double moller_sigma(double t, double tc) {
    if (!(t > 2.0 * tc)) return 0.0;
    const double tau = t / kMe, gamma = 1.0 + tau, b2 = 1.0 - 1.0 / (gamma * gamma);
    const double ec = tc / t, a = tau / gamma;
    const double br = 1.0 / ec - 1.0 / (1.0 - ec) + a * a * (0.5 - ec) -
                      (2.0 * tau + 1.0) / (gamma * gamma) * std::log((1.0 - ec) / ec);
    return kNa * kZoverA * 2.0 * kPi * kRe * kRe * kMe / (b2 * t) * br;
}

// k dsigma/dk of bremsstrahlung in water per unit density (cm^2/g): the
// Bethe-Heitler Born spectrum without screening (Koch and Motz formula 3BN),
// Z^2 replaced by the molecule's sum of Z (Z + 1); energies in mc^2 inside.
double brem_kdsig(double t, double k_mev) {
    const double e0 = 1.0 + t / kMe, k = k_mev / kMe, e = e0 - k;
    if (!(k > 0.0) || !(e > 1.0)) return 0.0;
    const double p0 = std::sqrt(e0 * e0 - 1.0), p = std::sqrt(e * e - 1.0);
    const double L = 2.0 * std::log((e0 * e + p0 * p - 1.0) / k);
    const double l0 = std::log((e0 + p0) / (e0 - p0)), l = std::log((e + p) / (e - p));
    const double p02 = p0 * p0, p2 = p * p, p03 = p02 * p0, p3 = p2 * p;
    const double br = 4.0 / 3.0 - 2.0 * e0 * e * (p2 + p02) / (p2 * p02) + l0 * e / p03 +
                      l * e0 / p3 - l * l0 / (p0 * p) +
                      L * (8.0 * e0 * e / (3.0 * p0 * p) + k * k * (e0 * e0 * e * e + p02 * p2) / (p03 * p3) +
                           k / (2.0 * p0 * p) *
                               (l0 * (e0 * e + p02) / p03 - l * (e0 * e + p2) / p3 +
                                2.0 * k * e0 * e / (p2 * p02)));
    const double v = (p / p0) * br;
    return v > 0.0 ? kZZ1Water * kAlphaFs * kRe * kRe * kNa / 18.0153 * v : 0.0;
}

// The continuous stopping power the range tables integrate: Bethe, or with
// the hard events on, the restricted collision part plus the radiative loss
// to photons below kc (`soft`, tabulated on log-spaced nodes and linear in
// ln T between them: at these cut-offs it is below 1e-3 of the total).
struct ContStop {
    bool dens = false, restrict_col = false;
    double tcut = 0.0;
    std::vector<double> soft;   // at exp(ls0 + i dls)
    double ls0 = 0.0, dls = 1.0;
    double operator()(double t) const {
        double s = restrict_col ? bethe_restricted(t, tcut, dens) : bethe(t, dens);
        if (!soft.empty()) {
            double x = (std::log(t) - ls0) / dls;
            x = std::min(std::max(x, 0.0), double(soft.size() - 1) - 1e-9);
            const int i = int(x);
            s += soft[i] + (x - i) * (soft[i + 1] - soft[i]);
        }
        return s;
    }
};

// Simpson integral of 1/S over [a, b] with m (even) panels; with the density
// effect the integrand has a kink where delta leaves zero (x0) and another at
// x1, and an interval across one is split there.
double inv_s_integral(double a, double b, int m, const ContStop& S) {
    if (S.dens) {
        for (double k : {t_at_x(kX0), t_at_x(kX1)})
            if (a < k && k < b) return inv_s_integral(a, k, m, S) + inv_s_integral(k, b, m, S);
    }
    const double h = (b - a) / m;
    double s = 1.0 / S(a) + 1.0 / S(b);
    for (int i = 1; i < m; ++i) s += (i % 2 ? 4.0 : 2.0) / S(a + i * h);
    return s * h / 3.0;
}

// ---- optional photon processes (water) --------------------------------------
constexpr double kAlpha = 7.2973525693e-3;
constexpr double kBohr = 0.529177210903e-8;     // cm
constexpr double kRydberg = 13.605693122994e-6; // MeV
constexpr double kHbarC = 1.973269804e-11;      // MeV cm
constexpr double kZeta3 = 1.2020569031595942;
constexpr double kMolPerGram = kNa / 18.0153;
constexpr double kZ1s = 7.70, kZn2 = 4.55;      // Slater-screened charges of O
constexpr double kRayTLo = 1.0e-4, kRayTHi = 4.0e8;   // t = (q a0)^2 nodes

// Stobbe: photoeffect of one hydrogenic K electron of nuclear charge z (cm^2).
double k_shell_electron(double e, double z) {
    const double ib = z * z * kRydberg;
    if (e <= ib) return 0.0;
    const double nu = std::sqrt(ib / (e - ib));
    const double x = ib / e, x2 = x * x;
    const double len = kBohr / z;
    const double coulomb = std::exp(-4.0 * nu * std::atan2(1.0, nu)) / -std::expm1(-2.0 * kPi * nu);
    return (512.0 / 3.0) * kPi * kPi * kAlpha * len * len * x2 * x2 * coulomb;
}

// Squared form factor of H2O (independent hydrogenic atoms) at t = (q a0)^2.
double water_ff2(double t) {
    auto f1s = [](double s2) { const double a = 1.0 + 0.25 * s2; return 1.0 / (a * a); };
    auto f2 = [](double s2, double num) {
        const double d = (1.0 + s2) * (1.0 + s2);
        return num / (d * d);
    };
    const double sa = t / (kZ1s * kZ1s), sb = t / (kZn2 * kZn2);
    const double hydrogen = f1s(t);
    const double oxygen = 2.0 * f1s(sa) + 2.0 * f2(sb, 1.0 - 3.0 * sb + 2.0 * sb * sb) +
                          4.0 * f2(sb, 1.0 - sb);
    return 2.0 * hydrogen * hydrogen + oxygen * oxygen;
}

// Unscreened Bethe-Heitler pair cross-section per unit Z^2 (Maximon).
double pair_per_z2(double e) {
    const double k = e / kMe;
    if (k <= 2.0) return 0.0;
    const double ar2 = kAlpha * kRe * kRe;
    if (k < 4.0) {
        const double ep = (2.0 * k - 4.0) / (2.0 + k + 2.0 * std::sqrt(2.0 * k));
        const double r = (k - 2.0) / k;
        const double series = 1.0 + ep * (0.5 + ep * (23.0 / 40.0 + ep * (11.0 / 60.0 + ep * 29.0 / 960.0)));
        return (2.0 * kPi / 3.0) * ar2 * r * r * r * series;
    }
    const double l = std::log(2.0 * k), y = 4.0 / (k * k);
    const double c2 = 6.0 * l - 3.5 + (2.0 / 3.0) * l * l * l - l * l - kPi * kPi / 3.0 * l +
                      2.0 * kZeta3 + kPi * kPi / 6.0;
    const double c4 = (3.0 / 16.0) * l + 0.125;
    const double c6 = (29.0 / 2304.0) * l - 77.0 / 13824.0;
    return ar2 * ((28.0 / 9.0) * l - 218.0 / 27.0 + y * c2 - y * y * c4 - y * y * y * c6);
}

// Integral of g over [a, b] (0 < a < b) by Simpson's rule in ln t.
template <class G>
double log_simpson(G&& g, double a, double b, int m) {
    const double la = std::log(a), h = (std::log(b) - la) / m;
    double s = 0.0;
    for (int i = 0; i <= m; ++i) {
        const double t = std::exp(la + i * h);
        const double w = (i == 0 || i == m) ? 1.0 : (i % 2 ? 4.0 : 2.0);
        s += w * g(t) * t;
    }
    return s * h / 3.0;
}

// Rayleigh cross-section of one molecule (cm^2) at photon energy e.
double rayleigh_molecule(double e) {
    const double x2 = (e * kBohr / kHbarC) * (e * kBohr / kHbarC);
    const double tmax = 4.0 * x2;
    auto g = [&](double t) {
        const double c = 1.0 - t / (2.0 * x2);
        return (1.0 + c * c) * water_ff2(t);
    };
    // [0, t1] with t1 tiny: F^2 and the angular factor are flat there
    const double t1 = std::min(1e-6, tmax);
    double sum = g(0.0) * t1;
    if (tmax > t1) sum += log_simpson(g, t1, tmax, 4000);
    return kPi * kRe * kRe / (2.0 * x2) * sum;
}

}  // namespace

void ensure_physics(psl_phantom* ph, const psl_transport_params* p) {
    PSL_CHECK(p->density_effect == 0 || p->density_effect == 1, "density_effect must be 0 or 1");
    const bool dens = p->density_effect == 1;
    PSL_CHECK((p->physics & ~(kPhysPhoto | kPhysRayleigh | kPhysPair | kPhysDelta | kPhysBrem)) == 0,
              "physics: unknown process bits 0x%x", p->physics);
    const uint32_t hard = p->physics & (kPhysDelta | kPhysBrem);
    PSL_CHECK(!(hard & kPhysBrem) || (p->e_cut_photon > 1e-3f && p->e_cut_photon < p->e_cut_electron * 50.f),
              "bremsstrahlung needs e_cut_photon in (0.001 MeV, 50 e_cut_electron)");
    PSL_CHECK(!(p->physics & kPhysPair) || p->e_cut_electron <= float(kMe),
              "pair production needs e_cut_electron <= mc^2 (every push then costs the "
              "photon at least the cut-off)");
    const float kc_key = (hard & kPhysBrem) ? p->e_cut_photon : 0.f;
    if (ph->t_cut_tab == p->e_cut_electron && ph->dens_tab == p->density_effect &&
        ph->phys_tab == int32_t(p->physics) && ph->kc_tab == kc_key && ph->tabs.p)
        return;
    const double tcut = p->e_cut_electron;
    PSL_CHECK(tcut > 2.0e-3 && tcut < 10.0, "e_cut_electron must be in (0.002, 10) MeV");
    // A photon pays at least the cut-off for every electron it sets in
    // motion, and the electron's random sub-stream id (1 + its push index)
    // has 8 bits in the particle tag: photons up to the top of the tables
    // must not push more than 255 electrons.
    PSL_CHECK(std::floor(kEmax / tcut) <= 255.0,
              "e_cut_electron must be at least %.4f MeV (at most 255 electrons per photon of "
              "up to %.0f MeV)", kEmax / 255.0, kEmax);

    const uint32_t phys = p->physics;
    // layout: kn, rng, inv, then (optional processes) xs as float4 (kept
    // 16-byte aligned), ray_t, ray_a, then (electron hard events) the hard
    // cross-sections as float2
    const size_t base = size_t(KN_TAB_N) + RNG_TAB_N + INV_TAB_N;
    const size_t extra = phys ? size_t(4) * KN_TAB_N + 2 * RAY_TAB_N : 0;
    const size_t extra_h = hard ? size_t(2) * RNG_TAB_N : 0;
    std::vector<float> host(base + extra + extra_h);
    float* kn = host.data();
    float* rng = kn + KN_TAB_N;
    float* inv = rng + RNG_TAB_N;

    const double ne = kNa * kZoverA;
    const double le0 = std::log(kEmin), dle = (std::log(kEmax) - le0) / (KN_TAB_N - 1);
    for (int i = 0; i < KN_TAB_N; ++i) kn[i] = float(ne * klein_nishina(std::exp(le0 + i * dle)));

    // the continuous stopping power
    ContStop S;
    S.dens = dens;
    S.restrict_col = (hard & kPhysDelta) != 0u;
    S.tcut = tcut;
    const double kc = p->e_cut_photon;
    if (hard & kPhysBrem) {
        const int ns = 256;
        S.ls0 = std::log(tcut);
        S.dls = (std::log(kTmax) - S.ls0) / (ns - 1);
        S.soft.resize(ns);
        for (int i = 0; i < ns; ++i) {
            const double t = std::exp(S.ls0 + i * S.dls), top = std::min(kc, t);
            S.soft[i] = log_simpson([&](double k) { return brem_kdsig(t, k); }, top * 1e-12, top, 400);
        }
    }
    // fine FP64 range table on a log grid, 16 Simpson panels per interval
    const int fine = 16 * (RNG_TAB_N - 1) + 1;
    const double lt0 = std::log(tcut), dlf = (std::log(kTmax) - lt0) / (fine - 1);
    std::vector<double> tf(fine), rf(fine);
    tf[0] = tcut;
    rf[0] = 0.0;
    for (int i = 1; i < fine; ++i) {
        tf[i] = std::exp(lt0 + i * dlf);
        rf[i] = rf[i - 1] + inv_s_integral(tf[i - 1], tf[i], 8, S);
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
            const double rt = rf[k] + inv_s_integral(tf[k], t, 8, S);
            t -= (rt - r) * S(t);
        }
        inv[i] = float(t);
    }
    double ray_lt1 = 0.0, ray_dlt = 1.0;
    if (phys) {
        float* xs = inv + INV_TAB_N;
        float* ray_t = xs + 4 * KN_TAB_N;
        float* ray_a = ray_t + RAY_TAB_N;
        for (int i = 0; i < KN_TAB_N; ++i) {
            const double e = std::exp(le0 + i * dle);
            const double mc = ne * klein_nishina(e);
            const double mp = (phys & kPhysPhoto) ? kMolPerGram * 2.0 * k_shell_electron(e, kZ1s) : 0.0;
            const double mr = (phys & kPhysRayleigh) ? kMolPerGram * rayleigh_molecule(e) : 0.0;
            const double mx = (phys & kPhysPair) ? kMolPerGram * 66.0 * pair_per_z2(e) : 0.0;
            xs[4 * i + 0] = float(mc);
            xs[4 * i + 1] = float(mc + mp);
            xs[4 * i + 2] = float(mc + mp + mr);
            xs[4 * i + 3] = float(mc + mp + mr + mx);
        }
        // t nodes: 0, then log-spaced from kRayTLo to kRayTHi; the cumulative
        // of F^2 between nodes by Simpson's rule in ln t
        ray_lt1 = std::log(kRayTLo);
        ray_dlt = (std::log(kRayTHi) - ray_lt1) / (RAY_TAB_N - 2);
        double acc = water_ff2(0.0) * kRayTLo;   // F^2 is flat below kRayTLo
        ray_t[0] = 0.f;
        ray_a[0] = 0.f;
        double prev = kRayTLo;
        ray_t[1] = float(kRayTLo);
        ray_a[1] = float(acc);
        for (int i = 2; i < RAY_TAB_N; ++i) {
            const double t = std::exp(ray_lt1 + (i - 1) * ray_dlt);
            acc += log_simpson(water_ff2, prev, t, 16);
            ray_t[i] = float(t);
            ray_a[i] = float(acc);
            prev = t;
        }
    }
    if (hard) {
        // hard-event cross-sections at the range table's nodes
        float* hx = host.data() + base + extra;
        for (int i = 0; i < RNG_TAB_N; ++i) {
            const double t = std::exp(lt0 + i * 16 * dlf);
            const double sm = (hard & kPhysDelta) ? moller_sigma(t, tcut) : 0.0;
            const double sbr = (hard & kPhysBrem) && t > kc
                                   ? log_simpson([&](double k) { return brem_kdsig(t, k) / k; }, kc, t, 400)
                                   : 0.0;
            hx[2 * i + 0] = float(sm);
            hx[2 * i + 1] = float(sm + sbr);
        }
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
    d.physics = phys;
    d.xs = phys ? reinterpret_cast<const float4*>(d.inv + INV_TAB_N) : nullptr;
    d.ray_t = phys ? d.inv + INV_TAB_N + 4 * KN_TAB_N : nullptr;
    d.ray_a = phys ? d.ray_t + RAY_TAB_N : nullptr;
    d.ray_lt1 = float(ray_lt1);
    d.ray_inv_dlt = float(1.0 / ray_dlt);
    d.ka0_per_mev = float(kBohr / kHbarC);
    d.photo_bind = float(kZ1s * kZ1s * kRydberg);
    d.hard = hard ? reinterpret_cast<const float2*>(d.kn + base + extra) : nullptr;
    ph->kc_tab = kc_key;
    ph->t_cut_tab = p->e_cut_electron;
    ph->dens_tab = p->density_effect;
    ph->phys_tab = int32_t(phys);
    ++ph->tab_gen;
}

}  // namespace psl
