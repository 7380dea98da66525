/*
 * physics.c -- oracle closed-form physics and tables. Test infrastructure only
 * (see omc_oracle.h).
 *
 * The paper (Sec. 2.1) takes photon data from NIST XCOM and electron data from
 * analytical formulae, tabulated per material. XCOM is not available, so every
 * quantity here is a closed form evaluated in FP64 and tabulated on 512 nodes
 * uniform in log2 E over [0.01, 20] MeV; lookups interpolate linearly in log2 E
 * (the paper uses hardware image interpolation, Sec. 2.2.2).
 *
 * Units: MeV, cm, g. Cross sections per gram are cm^2/g.
 */
#include <math.h>
#include <stdlib.h>
#include "omc_oracle.h"
#include "internal.h"

#define MC2 0.51099895
#define RE 2.8179403262e-13
#define ALPHA 7.2973525693e-3
#define NAV 6.02214076e23
#define PI 3.14159265358979323846

/* --- energy grid ------------------------------------------------------------ */
static double grid_L0(void) { return log2(ORC_ELO); }
static double grid_DL(void) { return log2(ORC_EHI / ORC_ELO) / (double)(ORC_NE - 1); }
static double grid_INV(void) { return (double)(ORC_NE - 1) / log2(ORC_EHI / ORC_ELO); }

double orc_node_energy(int i) { return exp2(grid_L0() + (double)i * grid_DL()); }

/* --- photons (Sec. 2.1: Compton, photoelectric, pair) ----------------------- */

/* Klein-Nishina total cross section per free electron, k = E/mc^2. */
double orc_sigma_kn(double E)
{
    const double k = E / MC2;
    const double l = log(1.0 + 2.0 * k);
    const double a = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k);
    const double b = l / (2.0 * k);
    const double c = (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
    return 2.0 * PI * RE * RE * (a + b - c);
}

/* Photoelectric absorption: non-relativistic Born K-shell form (Heitler)
 * sigma_K = 4 sqrt(2) Z^5 alpha^4 sigma_Thomson (mc^2/E)^(7/2), times 5/4 for the
 * outer shells. A rough stand-in for XCOM. */
double orc_sigma_pe_atom(int Z, double E)
{
    const double sigT = 8.0 * PI * RE * RE / 3.0;
    const double z5 = pow((double)Z, 5.0);
    const double a4 = pow(ALPHA, 4.0);
    return 1.25 * sigT * 4.0 * sqrt(2.0) * z5 * a4 * pow(MC2 / E, 3.5);
}

/* Pair production (only roughly modelled in Sec. 2.1): Maximon's near-threshold
 * Born series in the nuclear field, with Z(Z+1) to include the electron field. */
double orc_sigma_pair_atom(int Z, double E)
{
    const double k = E / MC2;
    if (k <= 2.0) return 0.0;
    const double e = (2.0 * k - 4.0) / (2.0 + k + 2.0 * sqrt(2.0 * k));
    const double r = (k - 2.0) / k;
    const double series = 1.0 + e / 2.0 + 23.0 * e * e / 40.0 + 11.0 * e * e * e / 60.0
                          + 29.0 * e * e * e * e / 960.0;
    return (2.0 * PI / 3.0) * ALPHA * RE * RE * (double)Z * (double)(Z + 1) * r * r * r * series;
}

static double electrons_per_gram(const orc_material* m)
{
    double s = 0.0;
    for (int j = 0; j < m->n_elem; ++j) s += m->w[j] * (double)m->Z[j] / m->A[j];
    return NAV * s;
}

static double mass_mu_compton(const orc_material* m, double E)
{
    return electrons_per_gram(m) * orc_sigma_kn(E);
}

static double mass_mu_pe(const orc_material* m, double E)
{
    double s = 0.0;
    for (int j = 0; j < m->n_elem; ++j) s += m->w[j] / m->A[j] * orc_sigma_pe_atom(m->Z[j], E);
    return NAV * s;
}

static double mass_mu_pair(const orc_material* m, double E)
{
    double s = 0.0;
    for (int j = 0; j < m->n_elem; ++j) s += m->w[j] / m->A[j] * orc_sigma_pair_atom(m->Z[j], E);
    return NAV * s;
}

/* --- electrons (Sec. 2.1: restricted stopping power, Moller, bremsstrahlung) - */

/* Restricted collision stopping power (Bethe with Moller cut Wcc), density
 * effect in its high-energy (Fermi) asymptote. */
double orc_scol_restricted(const orc_material* m, double T, double Wcc)
{
    const double tau = T / MC2;
    const double g = tau + 1.0;
    const double beta2 = tau * (tau + 2.0) / (g * g);
    double D = Wcc / MC2;
    if (D > tau / 2.0) D = tau / 2.0;
    const double Im = m->I_eV * 1e-6 / MC2;
    const double ZA = electrons_per_gram(m) / NAV;
    const double Fm = -1.0 - beta2 + log((tau - D) * D) + tau / (tau - D)
                      + (D * D / 2.0 + (2.0 * tau + 1.0) * log(1.0 - D / tau)) / (g * g);
    const double hw = 28.816 * sqrt(m->rho_nom * ZA); /* plasma energy, eV */
    double delta = 2.0 * log(sqrt(tau * (tau + 2.0))) + 2.0 * log(hw / m->I_eV) - 1.0;
    if (delta < 0.0) delta = 0.0;
    const double L = log(2.0 * (tau + 2.0) / (Im * Im)) + Fm - delta;
    return 2.0 * PI * RE * RE * MC2 * NAV * ZA / beta2 * L;
}

/* Radiation length of one element (Tsai), returned as 1/X0 in cm^2/g. */
double orc_inv_X0_element(int Z, double A)
{
    double Lrad, Lp;
    switch (Z) {
    case 1: Lrad = 5.31; Lp = 6.144; break;
    case 2: Lrad = 4.79; Lp = 5.621; break;
    case 3: Lrad = 4.74; Lp = 5.805; break;
    case 4: Lrad = 4.71; Lp = 5.924; break;
    default:
        Lrad = log(184.15 * pow((double)Z, -1.0 / 3.0));
        Lp = log(1194.0 * pow((double)Z, -2.0 / 3.0));
    }
    const double a = ALPHA * (double)Z;
    const double a2 = a * a;
    const double f = a2 * (1.0 / (1.0 + a2) + 0.20206 - 0.0369 * a2 + 0.0083 * a2 * a2
                           - 0.002 * a2 * a2 * a2);
    return 4.0 * ALPHA * RE * RE * NAV / A * ((double)Z * (double)Z * (Lrad - f) + (double)Z * Lp);
}

double orc_material_inv_X0(const orc_material* m)
{
    double s = 0.0;
    for (int j = 0; j < m->n_elem; ++j) s += m->w[j] * orc_inv_X0_element(m->Z[j], m->A[j]);
    return s;
}

/* Photon spectrum dsigma/dk = (1/X0)(1/k)(4/3 - 4/3 y + y^2), y = k/T, 0 < k <= T.
 * Restricted radiative loss: photons below kc stay in the continuous loss. */
double orc_srad_restricted(const orc_material* m, double T, double kc)
{
    const double ix0 = orc_material_inv_X0(m);
    const double k = kc < T ? kc : T;
    return ix0 * (4.0 * k / 3.0 - 2.0 * k * k / (3.0 * T) + k * k * k / (3.0 * T * T));
}

/* Hard bremsstrahlung (k > kc) per gram. */
double orc_sigma_brems(const orc_material* m, double T, double kc)
{
    if (T <= kc) return 0.0;
    const double ix0 = orc_material_inv_X0(m);
    const double r = kc / T;
    return ix0 * (4.0 / 3.0 * log(T / kc) - 4.0 / 3.0 * (1.0 - r) + (1.0 - r * r) / 2.0);
}

/* Hard Moller (energy transfer W > Wcc) per gram: the Moller cross section
 * per electron integrated over eps = W/T in [Wcc/T, 1/2]. */
double orc_sigma_moller(const orc_material* m, double T, double Wcc)
{
    if (T <= 2.0 * Wcc) return 0.0;
    const double tau = T / MC2;
    const double g = tau + 1.0;
    const double beta2 = tau * (tau + 2.0) / (g * g);
    const double e0 = Wcc / T;
    const double a = tau / g;
    const double b = (2.0 * tau + 1.0) / (g * g);
    const double I = 1.0 / e0 - 1.0 / (1.0 - e0) + a * a * (0.5 - e0) - b * log((1.0 - e0) / e0);
    return electrons_per_gram(m) * 2.0 * PI * RE * RE * MC2 / (beta2 * T) * I;
}

/* Transport (first-moment) cross section per gram for screened Rutherford
 * scattering with Moliere's screening parameter. */
double orc_K1(const orc_material* m, double T)
{
    const double pc2 = T * (T + 2.0 * MC2);
    const double g = T / MC2 + 1.0;
    const double beta2 = pc2 / (MC2 * MC2 * g * g);
    double s = 0.0;
    for (int j = 0; j < m->n_elem; ++j) {
        const double Z = (double)m->Z[j];
        const double aZ = ALPHA * Z;
        const double q = ALPHA * MC2 / (0.885 * sqrt(pc2));
        const double eta = 0.25 * q * q * pow(Z, 2.0 / 3.0) * (1.13 + 3.76 * aZ * aZ / beta2);
        const double sig1 = 2.0 * PI * Z * (Z + 1.0) * RE * RE * MC2 * MC2 / (beta2 * pc2)
                            * (log(1.0 + 1.0 / eta) - 1.0 / (1.0 + eta));
        s += m->w[j] / m->A[j] * sig1;
    }
    return NAV * s;
}

/* Mean of (1 - cos theta) for p(mu) ~ 1/(1 - mu + 2A)^2 on [-1, 1]. */
double orc_ms_m1(double A)
{
    return 2.0 * A * ((1.0 + A) * log1p(1.0 / A) - 1.0);
}

/* --- Gauss-Legendre nodes for the range integral -------------------------- */
static void gauss_legendre(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(PI * ((double)i + 0.75) / ((double)n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / (double)k;
                p0 = p1;
                p1 = p2;
            }
            dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute the derivative at the converged node */
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / (double)k;
            p0 = p1;
            p1 = p2;
        }
        dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

int orc_build_material(const orc_material* m, double Wcc, double kc, orc_mat_tables* t)
{
    if (!m || !t || m->n_elem <= 0) return -1;
    for (int i = 0; i < ORC_NE; ++i) {
        const double E = orc_node_energy(i);
        t->muC[i] = mass_mu_compton(m, E);
        t->muPE[i] = mass_mu_pe(m, E);
        t->muPair[i] = mass_mu_pair(m, E);
        t->muTot[i] = t->muC[i] + t->muPE[i] + t->muPair[i];
        t->Scol[i] = orc_scol_restricted(m, E, Wcc);
        t->Srad[i] = orc_srad_restricted(m, E, kc);
        t->sigM[i] = orc_sigma_moller(m, E, Wcc);
        t->sigB[i] = orc_sigma_brems(m, E, kc);
        t->K1[i] = orc_K1(m, E);
    }
    /* majorant for the hard-event Woodcock scheme: energy only decreases
     * within a step, so a running maximum over lower nodes bounds it */
    double run = 0.0;
    for (int i = 0; i < ORC_NE; ++i) {
        const double s = t->sigM[i] + t->sigB[i];
        if (s > run) run = s;
        t->sigHat[i] = run;
    }
    /* CSDA range: integral of dT/S_r from ELO, 16-point Gauss-Legendre in ln T
     * on each node interval, S_r from the closed forms */
    double gx[16], gw[16];
    gauss_legendre(16, gx, gw);
    t->R[0] = 0.0;
    for (int i = 0; i + 1 < ORC_NE; ++i) {
        const double a = log(orc_node_energy(i)), b = log(orc_node_energy(i + 1));
        const double hm = 0.5 * (b - a), c = 0.5 * (b + a);
        double s = 0.0;
        for (int j = 0; j < 16; ++j) {
            const double T = exp(c + hm * gx[j]);
            const double S = orc_scol_restricted(m, T, Wcc) + orc_srad_restricted(m, T, kc);
            s += gw[j] * T / S;
        }
        t->R[i + 1] = t->R[i] + hm * s;
    }
    return 0;
}

/* Screening parameter A as a function of x = s/lambda_1: the screened
 * Rutherford distribution whose mean (1 - cos) equals 1 - exp(-x), the exact
 * first moment after a path s (Goudsmit-Saunderson / Lewis). Solved by
 * bisection in ln A; tabulated as log2 A on nodes uniform in log2 x. */
void orc_build_ms_table(double* log2A)
{
    for (int j = 0; j < ORC_NA; ++j) {
        const double lx = ORC_XLO + (double)j * (ORC_XHI - ORC_XLO) / (double)(ORC_NA - 1);
        const double x = exp2(lx);
        const double target = -expm1(-x);
        double lo = log(1e-30), hi = log(1e12);
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (orc_ms_m1(exp(mid)) < target) lo = mid;
            else hi = mid;
        }
        log2A[j] = 0.5 * (lo + hi) / log(2.0);
    }
}

/* --- lookups --------------------------------------------------------------- */
void orc__grid_pos(double E, int* i, double* f)
{
    double t = (log2(E) - grid_L0()) * grid_INV();
    if (t < 0.0) t = 0.0;
    if (t > (double)(ORC_NE - 1)) t = (double)(ORC_NE - 1);
    int ii = (int)floor(t);
    if (ii > ORC_NE - 2) ii = ORC_NE - 2;
    *i = ii;
    *f = t - (double)ii;
}

double orc_table_lookup(const double* y, double E)
{
    int i;
    double f;
    orc__grid_pos(E, &i, &f);
    return y[i] + f * (y[i + 1] - y[i]);
}

double orc_range_inverse(const double* R, double Rv)
{
    if (Rv <= R[0]) return ORC_ELO;
    if (Rv >= R[ORC_NE - 1]) return ORC_EHI;
    int lo = 0, hi = ORC_NE - 1; /* R[lo] <= Rv < R[hi] */
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (R[mid] <= Rv) lo = mid;
        else hi = mid;
    }
    const double f = (Rv - R[lo]) / (R[lo + 1] - R[lo]);
    return exp2(grid_L0() + ((double)lo + f) * grid_DL());
}

double orc_ms_screening(const double* log2A, double x)
{
    double lx = log2(x);
    if (lx < ORC_XLO) lx = ORC_XLO;
    if (lx > ORC_XHI) lx = ORC_XHI;
    double t = (lx - ORC_XLO) * ((double)(ORC_NA - 1) / (ORC_XHI - ORC_XLO));
    int i = (int)floor(t);
    if (i > ORC_NA - 2) i = ORC_NA - 2;
    const double f = t - (double)i;
    return exp2(log2A[i] + f * (log2A[i + 1] - log2A[i]));
}
