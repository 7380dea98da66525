// tables.hpp -- host-side physics tables of the engine (FP64 closed forms).
//
// The paper (Sec. 2.1) keeps per-material photon attenuation per channel and
// electron restricted stopping power / hard cross sections, generated from an
// element composition. Here every quantity is a closed form evaluated in
// double precision on the host, tabulated on 512 nodes uniform in log2 E over
// [0.01, 20] MeV, then converted to the transport precision and staged in LDS
// by the kernels.
#pragma once

#include <array>
#include <vector>

namespace omc {

constexpr int kNE = 512;
constexpr double kELo = 0.01;
constexpr double kEHi = 20.0;
constexpr int kNA = 512;
constexpr double kXLo = -24.0;  // log2 of the smallest tabulated s/lambda_1
constexpr double kXHi = 3.0;    // log2 of the largest

constexpr double kMC2 = 0.51099895;          // electron rest energy, MeV
constexpr double kRe = 2.8179403262e-13;     // classical electron radius, cm
constexpr double kAlpha = 7.2973525693e-3;   // fine-structure constant
constexpr double kNA_ = 6.02214076e23;       // Avogadro
constexpr double kPi = 3.14159265358979323846;

struct Element {
    int Z;
    double A;
    double w;
};

struct MaterialSpec {
    std::vector<Element> elements;
    double I_eV = 75.0;
    double rho_nominal = 1.0;
};

// Energy grid: node i at log2 E = L0 + i * DL; a lookup uses
// t = (log2 E - L0) * INV, clamped to [0, NE-1].
struct EnergyGrid {
    double L0, DL, INV;
};
EnergyGrid energy_grid();
double node_energy(int i);

// Per-material tables in the order of omc_host_tables().
struct MaterialTables {
    std::array<double, kNE> muC, muPE, muPair, muTot, Scol, Srad, R, sigM, sigB, sigHat, K1;
};

MaterialTables build_material_tables(const MaterialSpec& m, double Wcc, double kc);
std::array<double, kNA> build_ms_table();

// Point evaluations (exposed for the engine's own checks).
double kn_cross_section(double E);
double restricted_collision_stopping(const MaterialSpec& m, double T, double Wcc);
double restricted_radiative_stopping(const MaterialSpec& m, double T, double kc);
double moller_hard(const MaterialSpec& m, double T, double Wcc);
double brems_hard(const MaterialSpec& m, double T, double kc);
double transport_xs(const MaterialSpec& m, double T);
double lerp_log2(const std::array<double, kNE>& y, double E);

}  // namespace omc
