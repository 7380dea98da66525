// tables.cpp -- closed-form physics of the engine, evaluated on the host in FP64.
//
// Photons (Sec. 2.1 of the paper: Compton, photoelectric, pair):
//   Compton       Klein-Nishina per free electron.
//   photoelectric Born K-shell form of Heitler, times 5/4 for outer shells
//                 (stand-in for the XCOM data the paper uses).
//   pair          Maximon's near-threshold Born series with Z(Z+1) for the
//                 electron field (the paper models pair production only roughly).
// Electrons (Sec. 2.1: restricted stopping power, Moller, bremsstrahlung):
//   collision     Bethe restricted to Moller transfers below Wcc, Fermi
//                 asymptote of the density effect.
//   radiative     Tsai radiation length; photon spectrum (1/k)(4/3 - 4/3 y + y^2),
//                 y = k/T: photons below kc are continuous loss, above kc hard.
//   Moller        integrated over eps = W/T in [Wcc/T, 1/2].
//   multiple      first transport cross section of screened Rutherford
//   scattering    scattering with Moliere screening; the screening parameter A
//                 of the step's angular distribution is matched to the exact
//                 first moment 1 - exp(-s/lambda_1).
#include "tables.hpp"

#include <cmath>

namespace omc {

EnergyGrid energy_grid()
{
    const double span = std::log2(kEHi / kELo);
    return EnergyGrid{std::log2(kELo), span / double(kNE - 1), double(kNE - 1) / span};
}

double node_energy(int i)
{
    const EnergyGrid g = energy_grid();
    return std::exp2(g.L0 + double(i) * g.DL);
}

namespace {

// electrons per gram / N_A  (sum of w Z / A)
double z_over_a(const MaterialSpec& m)
{
    double acc = 0.0;
    for (const Element& e : m.elements) acc += e.w * double(e.Z) / e.A;
    return acc;
}

template <class F>
double per_gram_atoms(const MaterialSpec& m, F sigma_atom)
{
    double acc = 0.0;
    for (const Element& e : m.elements) acc += e.w / e.A * sigma_atom(e.Z);
    return kNA_ * acc;
}

double pe_atom(int Z, double E)
{
    const double thomson = 8.0 * kPi * kRe * kRe / 3.0;
    return 1.25 * thomson * 4.0 * std::sqrt(2.0) * std::pow(double(Z), 5.0) *
           std::pow(kAlpha, 4.0) * std::pow(kMC2 / E, 3.5);
}

double pair_atom(int Z, double E)
{
    const double k = E / kMC2;
    if (k <= 2.0) return 0.0;
    const double eps = (2.0 * k - 4.0) / (2.0 + k + 2.0 * std::sqrt(2.0 * k));
    const double x = (k - 2.0) / k;
    const double poly = 1.0 + eps / 2.0 + 23.0 * eps * eps / 40.0 + 11.0 * eps * eps * eps / 60.0 +
                        29.0 * eps * eps * eps * eps / 960.0;
    return (2.0 * kPi / 3.0) * kAlpha * kRe * kRe * double(Z) * double(Z + 1) * x * x * x * poly;
}

double inv_rad_length_element(int Z, double A)
{
    // Tsai's L_rad and L'_rad; tabulated for the lightest elements
    static const double lrad_light[5] = {0.0, 5.31, 4.79, 4.74, 4.71};
    static const double lprime_light[5] = {0.0, 6.144, 5.621, 5.805, 5.924};
    const double z = double(Z);
    double lrad, lprime;
    if (Z <= 4) {
        lrad = lrad_light[Z];
        lprime = lprime_light[Z];
    } else {
        lrad = std::log(184.15 * std::pow(z, -1.0 / 3.0));
        lprime = std::log(1194.0 * std::pow(z, -2.0 / 3.0));
    }
    const double a2 = (kAlpha * z) * (kAlpha * z);
    const double coulomb =
        a2 * (1.0 / (1.0 + a2) + 0.20206 - 0.0369 * a2 + 0.0083 * a2 * a2 - 0.002 * a2 * a2 * a2);
    return 4.0 * kAlpha * kRe * kRe * kNA_ / A * (z * z * (lrad - coulomb) + z * lprime);
}

double inv_rad_length(const MaterialSpec& m)
{
    double acc = 0.0;
    for (const Element& e : m.elements) acc += e.w * inv_rad_length_element(e.Z, e.A);
    return acc;
}

// Gauss-Legendre abscissae and weights on [-1, 1] by Newton iteration on P_n.
void legendre_nodes(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    auto eval = [n](double z, double& p, double& dp) {
        double pm1 = 1.0, p0 = z;
        for (int k = 2; k <= n; ++k) {
            const double pk = ((2.0 * k - 1.0) * z * p0 - (k - 1.0) * pm1) / double(k);
            pm1 = p0;
            p0 = pk;
        }
        p = p0;
        dp = double(n) * (z * p0 - pm1) / (z * z - 1.0);
    };
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (double(i) + 0.75) / (double(n) + 0.5));
        for (int it = 0; it < 64; ++it) {
            double p, dp;
            eval(z, p, dp);
            const double step = p / dp;
            z -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        double p, dp;
        eval(z, p, dp);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

double ms_mean(double A)  // mean of 1 - cos for p ~ 1/(1 - cos + 2A)^2
{
    return 2.0 * A * ((1.0 + A) * std::log1p(1.0 / A) - 1.0);
}

}  // namespace

double kn_cross_section(double E)
{
    const double k = E / kMC2;
    const double q = 1.0 + 2.0 * k;
    const double lq = std::log(q);
    const double term1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / q - lq / k);
    const double term2 = lq / (2.0 * k);
    const double term3 = (1.0 + 3.0 * k) / (q * q);
    return 2.0 * kPi * kRe * kRe * (term1 + term2 - term3);
}

double restricted_collision_stopping(const MaterialSpec& m, double T, double Wcc)
{
    const double tau = T / kMC2;
    const double gam = tau + 1.0;
    const double b2 = tau * (tau + 2.0) / (gam * gam);
    const double delta_cut = std::fmin(Wcc / kMC2, 0.5 * tau);
    const double I = m.I_eV * 1e-6 / kMC2;
    const double za = z_over_a(m);
    const double fminus = -1.0 - b2 + std::log((tau - delta_cut) * delta_cut) +
                          tau / (tau - delta_cut) +
                          (0.5 * delta_cut * delta_cut + (2.0 * tau + 1.0) * std::log(1.0 - delta_cut / tau)) /
                              (gam * gam);
    const double plasma_eV = 28.816 * std::sqrt(m.rho_nominal * za);
    const double dens = std::fmax(
        0.0, 2.0 * std::log(std::sqrt(tau * (tau + 2.0))) + 2.0 * std::log(plasma_eV / m.I_eV) - 1.0);
    const double L = std::log(2.0 * (tau + 2.0) / (I * I)) + fminus - dens;
    return 2.0 * kPi * kRe * kRe * kMC2 * kNA_ * za / b2 * L;
}

double restricted_radiative_stopping(const MaterialSpec& m, double T, double kc)
{
    const double k = std::fmin(kc, T);
    return inv_rad_length(m) * (4.0 * k / 3.0 - 2.0 * k * k / (3.0 * T) + k * k * k / (3.0 * T * T));
}

double brems_hard(const MaterialSpec& m, double T, double kc)
{
    if (!(T > kc)) return 0.0;
    const double r = kc / T;
    return inv_rad_length(m) *
           (4.0 / 3.0 * std::log(T / kc) - 4.0 / 3.0 * (1.0 - r) + 0.5 * (1.0 - r * r));
}

double moller_hard(const MaterialSpec& m, double T, double Wcc)
{
    if (!(T > 2.0 * Wcc)) return 0.0;
    const double tau = T / kMC2;
    const double gam = tau + 1.0;
    const double b2 = tau * (tau + 2.0) / (gam * gam);
    const double e0 = Wcc / T;
    const double a = tau / gam;
    const double b = (2.0 * tau + 1.0) / (gam * gam);
    const double integral =
        1.0 / e0 - 1.0 / (1.0 - e0) + a * a * (0.5 - e0) - b * std::log((1.0 - e0) / e0);
    return kNA_ * z_over_a(m) * 2.0 * kPi * kRe * kRe * kMC2 / (b2 * T) * integral;
}

double transport_xs(const MaterialSpec& m, double T)
{
    const double pc2 = T * (T + 2.0 * kMC2);
    const double gam = T / kMC2 + 1.0;
    const double b2 = pc2 / (kMC2 * kMC2 * gam * gam);
    return per_gram_atoms(m, [&](int Zi) {
        const double z = double(Zi);
        const double q = kAlpha * kMC2 / (0.885 * std::sqrt(pc2));
        const double eta =
            0.25 * q * q * std::pow(z, 2.0 / 3.0) * (1.13 + 3.76 * (kAlpha * z) * (kAlpha * z) / b2);
        return 2.0 * kPi * z * (z + 1.0) * kRe * kRe * kMC2 * kMC2 / (b2 * pc2) *
               (std::log(1.0 + 1.0 / eta) - 1.0 / (1.0 + eta));
    });
}

MaterialTables build_material_tables(const MaterialSpec& m, double Wcc, double kc)
{
    MaterialTables t{};
    const double ne = kNA_ * z_over_a(m);
    for (int i = 0; i < kNE; ++i) {
        const double E = node_energy(i);
        t.muC[i] = ne * kn_cross_section(E);
        t.muPE[i] = per_gram_atoms(m, [E](int Z) { return pe_atom(Z, E); });
        t.muPair[i] = per_gram_atoms(m, [E](int Z) { return pair_atom(Z, E); });
        t.muTot[i] = t.muC[i] + t.muPE[i] + t.muPair[i];
        t.Scol[i] = restricted_collision_stopping(m, E, Wcc);
        t.Srad[i] = restricted_radiative_stopping(m, E, kc);
        t.sigM[i] = moller_hard(m, E, Wcc);
        t.sigB[i] = brems_hard(m, E, kc);
        t.K1[i] = transport_xs(m, E);
    }
    // majorant of the hard cross section for energies at or below each node
    double hi = 0.0;
    for (int i = 0; i < kNE; ++i) {
        hi = std::fmax(hi, t.sigM[i] + t.sigB[i]);
        t.sigHat[i] = hi;
    }
    // range: 16-point Gauss-Legendre in ln T over each node interval
    std::vector<double> gx, gw;
    legendre_nodes(16, gx, gw);
    t.R[0] = 0.0;
    for (int i = 1; i < kNE; ++i) {
        const double la = std::log(node_energy(i - 1)), lb = std::log(node_energy(i));
        const double half = 0.5 * (lb - la), mid = 0.5 * (lb + la);
        double acc = 0.0;
        for (int j = 0; j < 16; ++j) {
            const double T = std::exp(mid + half * gx[j]);
            acc += gw[j] * T /
                   (restricted_collision_stopping(m, T, Wcc) + restricted_radiative_stopping(m, T, kc));
        }
        t.R[i] = t.R[i - 1] + half * acc;
    }
    return t;
}

std::array<double, kNA> build_ms_table()
{
    std::array<double, kNA> out{};
    const double step = (kXHi - kXLo) / double(kNA - 1);
    for (int j = 0; j < kNA; ++j) {
        const double x = std::exp2(kXLo + double(j) * step);
        const double goal = -std::expm1(-x);  // exact first moment after s = x lambda_1
        // bisection on log2 A; m1(A) increases with A
        double lo = -100.0, hi = 40.0;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (ms_mean(std::exp2(mid)) < goal) lo = mid;
            else hi = mid;
        }
        out[j] = 0.5 * (lo + hi);
    }
    return out;
}

double lerp_log2(const std::array<double, kNE>& y, double E)
{
    const EnergyGrid g = energy_grid();
    double t = (std::log2(E) - g.L0) * g.INV;
    t = std::fmin(std::fmax(t, 0.0), double(kNE - 1));
    int i = int(std::floor(t));
    if (i > kNE - 2) i = kNE - 2;
    const double f = t - double(i);
    return y[i] + f * (y[i + 1] - y[i]);
}

}  // namespace omc
