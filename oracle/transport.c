/*
 * transport.c -- oracle coupled photon-electron transport. Test infrastructure
 * only (see omc_oracle.h): the GPU product path never calls this code.
 *
 * One history at a time, last-in-first-out over its particles (Sec. 2.2.1,
 * Table 1 describes the GPU scheduling; the physics of a particle does not
 * depend on the order because each particle owns its random stream).
 *
 *   photons   Sec. 2.1: Woodcock flights with the phantom majorant, real-event
 *             test, Compton (Klein-Nishina, Butcher-Messel sampling),
 *             photoelectric (local absorption), pair (e-/e+ along the photon,
 *             kinetic energy split uniformly).
 *   electrons Sec. 2.1: Class II condensed history; step
 *             d = min(d_vox, d_maxs, d_maxe, d_abs, d_event); random hinge with
 *             the multiple-scattering deflection (skipped for a step that ends
 *             on a face within the boundary skin); CSDA loss from the range table
 *             deposited in the voxel of the step; hard event accepted with the
 *             Woodcock ratio; Moller or bremsstrahlung; positrons annihilate
 *             into two back-to-back photons at the end of the track.
 *   tally     Sec. 2.2.2 (atomic dose counter) and Sec. 3.1 (sigma_D): energy
 *             per voxel per batch of histories, folded to dose (MeV/g per
 *             history) and the sum of squared batch doses.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>
#include "omc_oracle.h"
#include "internal.h"

#define MC2 0.51099895
#define PI 3.14159265358979323846

enum { LIM_VOX = 0, LIM_MAXS, LIM_MAXE, LIM_ABS, LIM_EVENT };
enum { PT_PHOTON = 0, PT_ELECTRON = 1, PT_POSITRON = 2 };

/* --- per-particle random stream --------------------------------------------- */
typedef struct {
    uint32_t key[2];
    uint64_t q;
    uint32_t n;  /* next block */
    int nw;      /* words of the cached block already used (4 = empty) */
    uint32_t w[4];
} rng_t;

static void rng_init(rng_t* r, uint32_t seed, uint32_t h, uint64_t q, uint32_t n0)
{
    r->key[0] = seed;
    r->key[1] = h;
    r->q = q;
    r->n = n0;
    r->nw = 4;
}

static uint32_t rng_word(rng_t* r)
{
    if (r->nw == 4) {
        const uint32_t ctr[4] = {r->n, (uint32_t)r->q, (uint32_t)(r->q >> 32), 0u};
        orc_philox4x32_10(ctr, r->key, r->w);
        r->n += 1;
        r->nw = 0;
    }
    return r->w[r->nw++];
}

static double rng_u(rng_t* r) { return orc_u01(rng_word(r)); }

/* A child's particle id: two raw words of the parent's stream, the high bit
 * set so that no child shares the source particle's id 0. */
static uint64_t rng_child_id(rng_t* r)
{
    const uint32_t lo = rng_word(r);
    const uint32_t hi = rng_word(r);
    return ((uint64_t)(hi | 0x80000000u) << 32) | (uint64_t)lo;
}

/* --- particles and the per-history stack ----------------------------------------- */
typedef struct {
    int type;
    double E;
    double x[3], d[3];
    int iv[3];
    double nmfp; /* remaining mean free paths to the next hard event; <0 unset */
    rng_t rng;
} part_t;

typedef struct {
    part_t* a;
    size_t n, cap;
} stack_t;

static void stack_push(stack_t* s, const part_t* p)
{
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 64;
        s->a = (part_t*)realloc(s->a, s->cap * sizeof(part_t));
    }
    s->a[s->n++] = *p;
}

/* --- run context ------------------------------------------------------------- */
typedef struct {
    const orc_problem* P;
    uint32_t seed;
    int n[3];
    double h[3];
    size_t nvox;
    double* rho;
    orc_mat_tables* tab;
    double* Rabs;  /* range at the electron absorption energy, per material */
    double muhat[ORC_NE];
    double log2A[ORC_NA];
    double* cdf;
    double skin; /* boundary skin depth, cm */
    /* macro cells of 2^cshift voxels per side (photon_mode 1): cn cells per
     * axis and the majorant scale q of each cell in 255ths */
    int cshift;
    int cn[3];
    unsigned char* cellq;
} ctx_t;

typedef struct {
    double* grid;
    orc_counters c;
} tally_t;

static size_t lin(const ctx_t* C, const int iv[3])
{
    return (size_t)iv[0] + (size_t)C->n[0] * ((size_t)iv[1] + (size_t)C->n[1] * (size_t)iv[2]);
}

static void deposit(tally_t* t, size_t v, double e)
{
    t->grid[v] += e;
    t->c.E_deposited += e;
}

static double lerp(const double* y, int i, double f) { return y[i] + f * (y[i + 1] - y[i]); }

/* Voxel containing x; 0 if outside the box. */
static int locate(const ctx_t* C, const double x[3], int iv[3])
{
    for (int a = 0; a < 3; ++a) {
        const double fl = floor(x[a] / C->h[a]);
        if (fl < 0.0 || fl >= (double)C->n[a]) return 0;
        iv[a] = (int)fl;
    }
    return 1;
}

/* Distance along d to the nearest face of voxel iv; ties go to the lower axis. */
static double dist_to_face(const ctx_t* C, const int iv[3], const double x[3], const double d[3],
                           int* axis)
{
    double best = INFINITY;
    int ax = 0;
    for (int a = 0; a < 3; ++a) {
        double s;
        if (d[a] > 0.0) s = ((double)(iv[a] + 1) * C->h[a] - x[a]) / d[a];
        else if (d[a] < 0.0) s = ((double)iv[a] * C->h[a] - x[a]) / d[a];
        else continue;
        if (s < best) {
            best = s;
            ax = a;
        }
    }
    if (best < 0.0) best = 0.0;
    *axis = ax;
    return best;
}

void orc_rotate(double d[3], double cost, double sint, double cphi, double sphi)
{
    const double u = d[0], v = d[1], w = d[2];
    const double r2 = 1.0 - w * w;
    if (r2 < 1e-12) {
        d[0] = sint * cphi;
        d[1] = sint * sphi;
        d[2] = w >= 0.0 ? cost : -cost;
        return;
    }
    const double r = sqrt(r2);
    d[0] = u * cost + sint * (u * w * cphi - v * sphi) / r;
    d[1] = v * cost + sint * (v * w * cphi + u * sphi) / r;
    d[2] = w * cost - sint * cphi * r;
}

/* --- samplers ------------------------------------------------------------------ */

/* Klein-Nishina by Butcher and Messel: eps = E'/E is drawn from the mixture of
 * 1/eps (weight a1) and eps (weight a2) on [eps0, 1] and accepted with
 * g = 1 - eps sin^2/(1 + eps^2). Returns eps, sets t = 1 - cos(theta). */
static double sample_compton_eps(rng_t* r, double k, double* t_out)
{
    const double e0 = 1.0 / (1.0 + 2.0 * k);
    const double a1 = log(1.0 + 2.0 * k);
    const double a2 = 0.5 * (1.0 - e0 * e0);
    for (;;) {
        const double ua = rng_u(r), ub = rng_u(r), uc = rng_u(r);
        double eps;
        if (ua * (a1 + a2) < a1) eps = exp(-a1 * ub);
        else eps = sqrt(e0 * e0 + (1.0 - e0 * e0) * ub);
        const double t = (1.0 - eps) / (k * eps);
        const double sin2 = t * (2.0 - t);
        if (uc <= 1.0 - eps * sin2 / (1.0 + eps * eps)) {
            *t_out = t;
            return eps;
        }
    }
}

/* Moller (Sec. 2.1: the energies from the cross section differential in
 * energy): eps = W/T on [eps0, 1/2] with density
 *   f(eps) = 1/eps^2 + 1/(1-eps)^2 + a^2 - b/(eps (1-eps)),
 * a = tau/(tau+1), b = (2 tau + 1)/(tau + 1)^2, tau = T/mc^2. The first three
 * terms, h(eps) >= f(eps), are a mixture with closed-form inverses: one
 * uniform picks the term by its integral over the interval, one samples eps
 * from it, and one accepts with probability f/h = 1 - b/(eps (1-eps) h). The
 * acceptance exceeds 99 % at 15 MeV and 55 % at the lowest energies. */
static double sample_moller_eps(rng_t* r, double T, double Wcc)
{
    const double e0 = Wcc / T;
    const double tau = T / MC2;
    const double g = tau + 1.0;
    const double a2 = (tau / g) * (tau / g);
    const double b = (2.0 * tau + 1.0) / (g * g);
    /* integrals of the three terms over [e0, 1/2] */
    const double w1 = 1.0 / e0 - 2.0;
    const double w2 = 2.0 - 1.0 / (1.0 - e0);
    const double w3 = a2 * (0.5 - e0);
    for (;;) {
        const double us = rng_u(r) * (w1 + w2 + w3);
        const double ue = rng_u(r);
        const double ua = rng_u(r);
        double eps;
        if (us < w1) eps = e0 / (1.0 - ue * (1.0 - 2.0 * e0));          /* 1/eps^2 */
        else if (us < w1 + w2) eps = 1.0 - 1.0 / (2.0 - ue * w2);     /* 1/(1-eps)^2 */
        else eps = e0 + ue * (0.5 - e0);                              /* a^2 */
        const double q = eps * (1.0 - eps);
        const double h = 1.0 / (eps * eps) + 1.0 / ((1.0 - eps) * (1.0 - eps)) + a2;
        if (ua * h <= h - b / q) return eps;
    }
}

/* Bremsstrahlung: k from 1/k on [kc, T], accepted with 1 - y + 0.75 y^2. */
static double sample_brems_k(rng_t* r, double T, double kc)
{
    const double lr = log(T / kc);
    for (;;) {
        const double ua = rng_u(r), ub = rng_u(r);
        const double k = kc * exp(ua * lr);
        const double y = k / T;
        if (ub <= 1.0 - y + 0.75 * y * y) return k;
    }
}

/* Screened-Rutherford deflection with screening A: 1 - cos = 2 A u/(1 + A - u). */
static double sample_ms(rng_t* r, double A)
{
    const double u = rng_u(r);
    return 2.0 * A * u / (1.0 + A - u);
}

/* The hinge deflection of a step: polar angle from the screened-Rutherford
 * form, azimuth uniform, applied to d; returns 1 - cos(theta). */
static double ms_deflect(rng_t* r, double A, double d[3])
{
    const double omc = sample_ms(r, A);
    const double phi = 2.0 * PI * rng_u(r);
    orc_rotate(d, 1.0 - omc, sqrt(omc * (2.0 - omc)), cos(phi), sin(phi));
    return omc;
}

/* --- secondaries ------------------------------------------------------------------ */
static void emit_photon(const ctx_t* C, stack_t* st, tally_t* t, rng_t* parent, double E,
                        const double x[3], const int iv[3], const double d[3]);

static void annihilate(const ctx_t* C, stack_t* st, tally_t* t, rng_t* r, const double x[3],
                       const int iv[3])
{
    t->c.pos_annihil++;
    t->c.E_annih_rest += 2.0 * MC2;
    const double c = 2.0 * rng_u(r) - 1.0;
    const double phi = 2.0 * PI * rng_u(r);
    const double s = sqrt((1.0 - c) * (1.0 + c));
    const double a[3] = {s * cos(phi), s * sin(phi), c};
    const double b[3] = {-a[0], -a[1], -a[2]};
    emit_photon(C, st, t, r, MC2, x, iv, a);
    emit_photon(C, st, t, r, MC2, x, iv, b);
}

static void emit_photon(const ctx_t* C, stack_t* st, tally_t* t, rng_t* parent, double E,
                        const double x[3], const int iv[3], const double d[3])
{
    if (E >= C->P->Eabs_g) {
        part_t c;
        c.type = PT_PHOTON;
        c.E = E;
        memcpy(c.x, x, sizeof c.x);
        memcpy(c.d, d, sizeof c.d);
        memcpy(c.iv, iv, sizeof c.iv);
        c.nmfp = -1.0;
        rng_init(&c.rng, C->seed, parent->key[1], rng_child_id(parent), 0u);
        stack_push(st, &c);
        t->c.push_ph++;
    } else {
        deposit(t, lin(C, iv), E);
    }
}

static void emit_electron(const ctx_t* C, stack_t* st, tally_t* t, rng_t* parent, int type,
                          double E, const double x[3], const int iv[3], const double d[3])
{
    if (!C->P->kerma_mode && E >= C->P->Eabs_e) {
        part_t c;
        c.type = type;
        c.E = E;
        memcpy(c.x, x, sizeof c.x);
        memcpy(c.d, d, sizeof c.d);
        memcpy(c.iv, iv, sizeof c.iv);
        c.nmfp = -1.0;
        rng_init(&c.rng, C->seed, parent->key[1], rng_child_id(parent), 0u);
        stack_push(st, &c);
        t->c.push_el++;
    } else {
        deposit(t, lin(C, iv), E);
        if (type == PT_POSITRON) annihilate(C, st, t, parent, x, iv);
    }
}

/* --- photons ----------------------------------------------------------------------- */

/* Woodcock flights until a real interaction; 0 if the photon left the box. */
static int woodcock(const ctx_t* C, part_t* p, tally_t* t, size_t* vout, int* iout, double* fout)
{
    int i;
    double f;
    orc__grid_pos(p->E, &i, &f);
    const double mh = lerp(C->muhat, i, f);
    for (;;) {
        const double s = -log(rng_u(&p->rng)) / mh;
        for (int a = 0; a < 3; ++a) p->x[a] = p->x[a] + s * p->d[a];
        t->c.ph_flights++;
        if (!locate(C, p->x, p->iv)) {
            t->c.E_escaped += p->E;
            t->c.ph_escaped++;
            return 0;
        }
        const size_t v = lin(C, p->iv);
        const orc_mat_tables* T = &C->tab[C->P->mat[v]];
        const double mt = lerp(T->muTot, i, f);
        if (rng_u(&p->rng) * mh < C->rho[v] * mt) {
            *vout = v;
            *iout = i;
            *fout = f;
            return 1;
        }
        t->c.ph_fictitious++;
    }
}

/* The same flights with a majorant per macro cell (photon_mode 1): the
 * optical depth tau = -ln u is spent cell by cell, mu_c = mu_hat * q_c / 255
 * in cell c, the path crossing each cell face (snapped onto it, the cell
 * index stepped); the candidate is accepted with rho mu / mu_c. Leaving the
 * cell grid or the box is an escape. Ties between faces go to the lower axis. */
static int woodcock_cells(const ctx_t* C, part_t* p, tally_t* t, size_t* vout, int* iout,
                          double* fout)
{
    int i;
    double f;
    orc__grid_pos(p->E, &i, &f);
    const double mh = lerp(C->muhat, i, f);
    const int S = C->cshift;
    const double W[3] = {(double)(1 << S) * C->h[0], (double)(1 << S) * C->h[1],
                         (double)(1 << S) * C->h[2]};
    const int maxn = C->cn[0] + C->cn[1] + C->cn[2] + 2;
    for (;;) {
        double tau = -log(rng_u(&p->rng));
        t->c.ph_flights++;
        int c[3] = {p->iv[0] >> S, p->iv[1] >> S, p->iv[2] >> S};
        double mc = mh;
        int inside = 0, left = 0;
        for (int n = 0; n < maxn; ++n) {
            const int q = C->cellq[c[0] + C->cn[0] * (c[1] + C->cn[1] * c[2])];
            mc = q == 255 ? mh : (mh * (double)q) / 255.0;
            double d = INFINITY;
            int ax = 0;
            for (int a = 0; a < 3; ++a) {
                double ta;
                if (p->d[a] > 0.0)
                    ta = ((double)(c[a] + 1) * W[a] - p->x[a]) / p->d[a];
                else if (p->d[a] < 0.0)
                    ta = ((double)c[a] * W[a] - p->x[a]) / p->d[a];
                else
                    continue;
                if (ta < d) {
                    d = ta;
                    ax = a;
                }
            }
            if (d < 0.0) d = 0.0;
            if (tau < mc * d) {
                const double s = tau / mc;
                for (int a = 0; a < 3; ++a) p->x[a] = p->x[a] + s * p->d[a];
                inside = 1;
                break;
            }
            tau = tau - mc * d;
            for (int a = 0; a < 3; ++a) p->x[a] = p->x[a] + d * p->d[a];
            const int up = p->d[ax] > 0.0;
            p->x[ax] = (double)(c[ax] + up) * W[ax];
            c[ax] += up ? 1 : -1;
            if (c[ax] < 0 || c[ax] >= C->cn[ax]) {
                left = 1;
                break;
            }
        }
        /* a straight line crosses at most cn[0] + cn[1] + cn[2] cell faces;
         * reaching the bound would be a rounding failure, not an escape */
        if (!inside && !left) t->c.watchdog++;
        if (!inside || !locate(C, p->x, p->iv)) {
            t->c.E_escaped += p->E;
            t->c.ph_escaped++;
            return 0;
        }
        const size_t v = lin(C, p->iv);
        const orc_mat_tables* T = &C->tab[C->P->mat[v]];
        const double mt = lerp(T->muTot, i, f);
        if (rng_u(&p->rng) * mc < C->rho[v] * mt) {
            *vout = v;
            *iout = i;
            *fout = f;
            return 1;
        }
        t->c.ph_fictitious++;
    }
}

/* Interaction type at a real event: 1 Compton, 2 photoelectric, 3 pair.
 * Below the pair threshold the pair interval counts as absorption. */
static int select_type(const ctx_t* C, part_t* p, size_t v, int i, double f)
{
    const orc_mat_tables* T = &C->tab[C->P->mat[v]];
    const double mt = lerp(T->muTot, i, f);
    const double sel = rng_u(&p->rng) * mt;
    const double mc = lerp(T->muC, i, f);
    const double mp = lerp(T->muPE, i, f);
    if (sel < mc) return 1;
    if (sel < mc + mp) return 2;
    if (p->E <= 2.0 * MC2) return 2;
    return 3;
}

static void compton(const ctx_t* C, part_t* p, stack_t* st, tally_t* t)
{
    const double E = p->E;
    const double k = E / MC2;
    double tt;
    const double eps = sample_compton_eps(&p->rng, k, &tt);
    const double sin2 = tt * (2.0 - tt);
    const double cost = 1.0 - tt;
    const double sint = sqrt(sin2 > 0.0 ? sin2 : 0.0);
    const double phi = 2.0 * PI * rng_u(&p->rng);
    const double d0[3] = {p->d[0], p->d[1], p->d[2]};
    orc_rotate(p->d, cost, sint, cos(phi), sin(phi));
    const double Ep = eps * E;
    const double Te = E - Ep;
    /* recoil electron: momentum balance E d0 = E' d + p_e */
    double pe[3];
    for (int a = 0; a < 3; ++a) pe[a] = E * d0[a] - Ep * p->d[a];
    const double nrm = sqrt(pe[0] * pe[0] + pe[1] * pe[1] + pe[2] * pe[2]);
    double de[3];
    for (int a = 0; a < 3; ++a) de[a] = nrm > 0.0 ? pe[a] / nrm : d0[a];
    t->c.ph_compton++;
    emit_electron(C, st, t, &p->rng, PT_ELECTRON, Te, p->x, p->iv, de);
    p->E = Ep;
}

static void pair(const ctx_t* C, part_t* p, stack_t* st, tally_t* t)
{
    const double K = p->E - 2.0 * MC2;
    const double Tm = rng_u(&p->rng) * K;
    const double Tp = K - Tm;
    t->c.ph_pair++;
    t->c.E_pair_rest += 2.0 * MC2;
    emit_electron(C, st, t, &p->rng, PT_ELECTRON, Tm, p->x, p->iv, p->d);
    emit_electron(C, st, t, &p->rng, PT_POSITRON, Tp, p->x, p->iv, p->d);
}

static void transport_photon(const ctx_t* C, part_t* p, stack_t* st, tally_t* t)
{
    for (;;) {
        if (p->E < C->P->Eabs_g) {
            deposit(t, lin(C, p->iv), p->E);
            t->c.ph_cutoff++;
            return;
        }
        size_t v;
        int i;
        double f;
        const int real = C->P->photon_mode == 1 ? woodcock_cells(C, p, t, &v, &i, &f)
                                                 : woodcock(C, p, t, &v, &i, &f);
        if (!real) return;
        const int type = select_type(C, p, v, i, f);
        if (type == 1) {
            compton(C, p, st, t);
        } else if (type == 2) {
            deposit(t, v, p->E);
            t->c.ph_photo++;
            return;
        } else {
            pair(C, p, st, t);
            return;
        }
    }
}

/* --- electrons and positrons -------------------------------------------------------- */

static void moller(const ctx_t* C, part_t* p, stack_t* st, tally_t* t)
{
    const double T = p->E;
    if (T <= 2.0 * C->P->Wcc) {
        t->c.el_hard_fict++;
        return;
    }
    const double eps = sample_moller_eps(&p->rng, T, C->P->Wcc);
    const double W = eps * T;
    const double Tp = T - W;
    const double cp = sqrt(Tp * (T + 2.0 * MC2) / (T * (Tp + 2.0 * MC2)));
    const double cd = sqrt(W * (T + 2.0 * MC2) / (T * (W + 2.0 * MC2)));
    const double sp = sqrt(1.0 - cp * cp > 0.0 ? 1.0 - cp * cp : 0.0);
    const double sd = sqrt(1.0 - cd * cd > 0.0 ? 1.0 - cd * cd : 0.0);
    const double phi = 2.0 * PI * rng_u(&p->rng);
    const double cf = cos(phi), sf = sin(phi);
    double dd[3] = {p->d[0], p->d[1], p->d[2]};
    orc_rotate(dd, cd, sd, -cf, -sf); /* azimuth phi + pi */
    orc_rotate(p->d, cp, sp, cf, sf);
    t->c.el_moller++;
    p->E = Tp;
    emit_electron(C, st, t, &p->rng, PT_ELECTRON, W, p->x, p->iv, dd);
}

static void brems(const ctx_t* C, part_t* p, stack_t* st, tally_t* t)
{
    const double T = p->E;
    if (T <= C->P->kc) {
        t->c.el_hard_fict++;
        return;
    }
    const double k = sample_brems_k(&p->rng, T, C->P->kc);
    const double th = MC2 / (T + MC2); /* angle of the maximum of the photon DCS */
    const double phi = 2.0 * PI * rng_u(&p->rng);
    double dg[3] = {p->d[0], p->d[1], p->d[2]};
    orc_rotate(dg, cos(th), sin(th), cos(phi), sin(phi));
    t->c.el_brems++;
    p->E = T - k;
    emit_photon(C, st, t, &p->rng, k, p->x, p->iv, dg);
}

/* Test hook (orc_first_hard): while active, voxel-limited electron steps add
 * their mass path rho*s to tau, and the first accepted hard-event candidate
 * records the energy there and its kind and ends the particle's transport.
 * One history at a time (single-threaded use only). */
static struct {
    int active, done, kind;
    double tau, T;
} g_first;

/* Candidate hard event at the end of an event-limited step: accepted with the
 * Woodcock ratio sigma(T_end)/sigma_hat(T_start) in mass units. */
static void hard_event(const ctx_t* C, part_t* p, const orc_mat_tables* T, double shm,
                       stack_t* st, tally_t* t)
{
    t->c.el_hard_cand++;
    int i;
    double f;
    orc__grid_pos(p->E, &i, &f);
    const double sM = lerp(T->sigM, i, f);
    const double sB = lerp(T->sigB, i, f);
    const double sH = sM + sB;
    if (rng_u(&p->rng) * shm < sH) {
        const int is_moller = rng_u(&p->rng) * sH < sM;
        if (g_first.active && !g_first.done) {
            g_first.done = 1;
            g_first.kind = is_moller ? 1 : 2;
            g_first.T = p->E;
        }
        if (is_moller) moller(C, p, st, t);
        else brems(C, p, st, t);
    } else {
        t->c.el_hard_fict++;
    }
    p->nmfp = -log(rng_u(&p->rng));
}

/* Step trace of one history (debugging aid, single-threaded use only). */
static double* g_trace = NULL;
static uint32_t g_trace_cap = 0, g_trace_n = 0;

static void trace_step(const ctx_t* C, const part_t* p, int code)
{
    if (!g_trace) return;
    if (g_trace_n < g_trace_cap) {
        double* r = g_trace + 12 * (size_t)g_trace_n;
        r[0] = code;
        r[1] = (double)(uint32_t)p->rng.q;
        r[2] = (double)(uint32_t)(p->rng.q >> 32);
        r[3] = 4.0 * (double)p->rng.n - (double)(4 - p->rng.nw);
        for (int a = 0; a < 3; ++a) {
            r[4 + a] = p->x[a];
            r[7 + a] = p->d[a];
        }
        r[10] = p->E;
        r[11] = (double)p->iv[0] + 1024.0 * ((double)p->iv[1] + 1024.0 * (double)p->iv[2]);
    }
    g_trace_n++;
    (void)C;
}

static void transport_electron(const ctx_t* C, part_t* p, stack_t* st, tally_t* t)
{
    const orc_problem* P = C->P;
    for (;;) {
        const size_t v = lin(C, p->iv);
        if (p->E <= P->Eabs_e) {
            deposit(t, v, p->E);
            t->c.el_absorbed++;
            trace_step(C, p, 64);
            if (p->type == PT_POSITRON) annihilate(C, st, t, &p->rng, p->x, p->iv);
            return;
        }
        const orc_mat_tables* T = &C->tab[P->mat[v]];
        const double rho = C->rho[v];
        if (!P->csda_mode && p->nmfp < 0.0) p->nmfp = -log(rng_u(&p->rng));
        const double T0 = p->E;
        int i;
        double f;
        orc__grid_pos(T0, &i, &f);
        const double RT = lerp(T->R, i, f);
        const double shm = lerp(T->sigHat, i, f);
        const double sig_hat = rho * shm;
        double d_event = INFINITY;
        if (!P->csda_mode && sig_hat > 0.0) d_event = p->nmfp / sig_hat;
        int ax;
        const double d_vox = dist_to_face(C, p->iv, p->x, p->d, &ax);
        const double d_maxs = P->dmax_s;
        const double d_maxe = (RT - orc_table_lookup(T->R, (1.0 - P->f_E) * T0)) / rho;
        const double d_abs = (RT - C->Rabs[P->mat[v]]) / rho;
        double d = d_vox;
        int lim = LIM_VOX;
        if (d_maxs < d) { d = d_maxs; lim = LIM_MAXS; }
        if (d_maxe < d) { d = d_maxe; lim = LIM_MAXE; }
        if (d_abs < d) { d = d_abs; lim = LIM_ABS; }
        if (d_event < d) { d = d_event; lim = LIM_EVENT; }

        int crossed = 0, cax = ax;
        if (d > 0.0) {
            double s;
            if (P->csda_mode || (lim == LIM_VOX && d < C->skin)) {
                /* straight line; inside the boundary skin the hinge deflection
                 * is skipped and the step ends on the face */
                for (int a = 0; a < 3; ++a) p->x[a] = p->x[a] + d * p->d[a];
                s = d;
                if (lim == LIM_VOX) crossed = 1;
            } else {
                /* random hinge: straight to xi*d, deflect, then the rest */
                const double xi = rng_u(&p->rng);
                const double s1 = xi * d;
                for (int a = 0; a < 3; ++a) p->x[a] = p->x[a] + s1 * p->d[a];
                const double Tplan = orc_range_inverse(T->R, RT - rho * d);
                const double Tmid = 0.5 * (T0 + Tplan);
                const double xs = d * rho * orc_table_lookup(T->K1, Tmid);
                const double A = orc_ms_screening(C->log2A, xs);
                ms_deflect(&p->rng, A, p->d);
                const double rem = (1.0 - xi) * d;
                int ax2;
                const double dv2 = dist_to_face(C, p->iv, p->x, p->d, &ax2);
                double s2 = rem;
                if (dv2 < rem) {
                    s2 = dv2;
                    crossed = 1;
                    cax = ax2;
                    t->c.el_hinge_trunc++;
                }
                for (int a = 0; a < 3; ++a) p->x[a] = p->x[a] + s2 * p->d[a];
                s = s1 + s2;
            }
            double Tend;
            if (lim == LIM_ABS && !crossed) Tend = P->Eabs_e;
            else Tend = orc_range_inverse(T->R, RT - rho * s);
            deposit(t, v, T0 - Tend);
            if (!P->csda_mode) {
                p->nmfp = p->nmfp - sig_hat * s;
                if (p->nmfp < 0.0) p->nmfp = 0.0;
            }
            t->c.el_steps++;
            p->E = Tend;
            if (g_first.active) g_first.tau += rho * s;
        } else if (lim == LIM_VOX) {
            crossed = 1; /* zero-length step on a face: only the index moves */
        } else if (lim == LIM_ABS) {
            /* no range left above the absorption energy (T within rounding of
             * E_abs): the track ends; the remainder is deposited here */
            deposit(t, v, T0 - P->Eabs_e);
            p->E = P->Eabs_e;
        }

        if (crossed) {
            const int a = cax;
            const int up = p->d[a] > 0.0;
            p->x[a] = up ? (double)(p->iv[a] + 1) * C->h[a] : (double)p->iv[a] * C->h[a];
            p->iv[a] += up ? 1 : -1;
            t->c.el_boundary++;
            trace_step(C, p, 16 + lim + 8 * crossed);
            if (p->iv[a] < 0 || p->iv[a] >= C->n[a]) {
                t->c.E_escaped += p->E;
                t->c.el_escaped++;
                return;
            }
            continue;
        }
        if (lim == LIM_EVENT) hard_event(C, p, T, shm, st, t);
        trace_step(C, p, 16 + lim);
        if (g_first.active && g_first.done) return;
    }
}

/* --- fixed-step electrons (the gDPM scheme of Sec. 4) --------------------------------
 *
 * Sec. 4 contrasts the voxel-limited step above with gDPM's fixed step, in which
 * an electron crosses voxel faces within a step and only a hard event (or the
 * other limits) ends it, relying on a scaling of the cross sections between
 * materials. Reading: a step is planned in mass thickness tau (g/cm^2) with the
 * mass stopping power, cross sections and transport coefficient of the material
 * of the voxel where it starts (m0), which stand for every material it crosses:
 * only the density changes along the step (density scaling). Limits:
 * tau_maxs = d_maxs x 1 g/cm^3 (a water-equivalent length), tau_maxe and
 * tau_abs from m0's range table, tau_event = n_mfp / sigma_hat(T0). The path,
 * with the random hinge at xi tau, is marched voxel by voxel: a voxel of
 * density rho consumes rho x length of tau, and the CSDA energy lost inside it,
 * T(R0 - tau_in) - T(R0 - tau_out), is deposited there. A step that leaves the
 * phantom ends the track (escape). */

/* Move along d until tau_done reaches `target`, depositing the CSDA loss per
 * voxel. Returns 1 if the particle leaves the phantom. end_abs: the step ends
 * at the absorption energy exactly. */
static int march(const ctx_t* C, part_t* p, tally_t* t, const orc_mat_tables* T, double RT,
                 double target, int end_abs, double* tau_done, double* Tcur)
{
    for (;;) {
        const size_t v = lin(C, p->iv);
        const double rho = C->rho[v];
        int ax;
        const double dface = dist_to_face(C, p->iv, p->x, p->d, &ax);
        const double rem = target - *tau_done;
        if (rem <= rho * dface) {
            const double s = rem / rho;
            for (int a = 0; a < 3; ++a) p->x[a] = p->x[a] + s * p->d[a];
            const double Tn = end_abs ? C->P->Eabs_e : orc_range_inverse(T->R, RT - target);
            deposit(t, v, *Tcur - Tn);
            *Tcur = Tn;
            *tau_done = target;
            return 0;
        }
        for (int a = 0; a < 3; ++a) p->x[a] = p->x[a] + dface * p->d[a];
        *tau_done = *tau_done + rho * dface;
        const double Tn = orc_range_inverse(T->R, RT - *tau_done);
        deposit(t, v, *Tcur - Tn);
        *Tcur = Tn;
        /* onto the face, index stepped (as for a voxel-limited crossing) */
        const int up = p->d[ax] > 0.0;
        p->x[ax] = up ? (double)(p->iv[ax] + 1) * C->h[ax] : (double)p->iv[ax] * C->h[ax];
        p->iv[ax] += up ? 1 : -1;
        t->c.el_boundary++;
        if (p->iv[ax] < 0 || p->iv[ax] >= C->n[ax]) return 1;
    }
}

static void transport_electron_fixed(const ctx_t* C, part_t* p, stack_t* st, tally_t* t)
{
    const orc_problem* P = C->P;
    for (;;) {
        const size_t v = lin(C, p->iv);
        if (p->E <= P->Eabs_e) {
            deposit(t, v, p->E);
            t->c.el_absorbed++;
            trace_step(C, p, 64);
            if (p->type == PT_POSITRON) annihilate(C, st, t, &p->rng, p->x, p->iv);
            return;
        }
        const int m0 = P->mat[v];
        const orc_mat_tables* T = &C->tab[m0];
        if (!P->csda_mode && p->nmfp < 0.0) p->nmfp = -log(rng_u(&p->rng));
        const double T0 = p->E;
        int i;
        double f;
        orc__grid_pos(T0, &i, &f);
        const double RT = lerp(T->R, i, f);
        const double shm = lerp(T->sigHat, i, f);
        double t_event = INFINITY;
        if (!P->csda_mode && shm > 0.0) t_event = p->nmfp / shm;
        const double t_maxs = P->dmax_s * 1.0; /* g/cm^2: d_maxs of unit density */
        const double t_maxe = RT - orc_table_lookup(T->R, (1.0 - P->f_E) * T0);
        const double t_abs = RT - C->Rabs[m0];
        double tau = t_maxs;
        int lim = LIM_MAXS;
        if (t_maxe < tau) { tau = t_maxe; lim = LIM_MAXE; }
        if (t_abs < tau) { tau = t_abs; lim = LIM_ABS; }
        if (t_event < tau) { tau = t_event; lim = LIM_EVENT; }

        if (tau > 0.0) {
            double done = 0.0, Tcur = T0;
            int out;
            if (P->csda_mode) {
                out = march(C, p, t, T, RT, tau, lim == LIM_ABS, &done, &Tcur);
            } else {
                const double xi = rng_u(&p->rng);
                out = march(C, p, t, T, RT, xi * tau, 0, &done, &Tcur);
                if (!out) {
                    const double Tplan = orc_range_inverse(T->R, RT - tau);
                    const double Tmid = 0.5 * (T0 + Tplan);
                    const double A = orc_ms_screening(C->log2A, tau * orc_table_lookup(T->K1, Tmid));
                    ms_deflect(&p->rng, A, p->d);
                    out = march(C, p, t, T, RT, tau, lim == LIM_ABS, &done, &Tcur);
                }
            }
            if (!P->csda_mode) {
                p->nmfp = p->nmfp - shm * done;
                if (p->nmfp < 0.0) p->nmfp = 0.0;
            }
            t->c.el_steps++;
            p->E = Tcur;
            if (out) {
                t->c.E_escaped += p->E;
                t->c.el_escaped++;
                trace_step(C, p, 16 + lim + 8);
                return;
            }
        } else if (lim == LIM_ABS) {
            deposit(t, v, T0 - P->Eabs_e);
            p->E = P->Eabs_e;
        }
        if (lim == LIM_EVENT) hard_event(C, p, T, shm, st, t);
        trace_step(C, p, 16 + lim);
    }
}

/* --- source (Sec. 2.2 "Materials": point source, SSD, field at the surface) --------- */

/* Draws block 0 of stream (seed, h, 0): u1,u2 energy, u3,u4 position.
 * Returns 0 when the ray misses the phantom. */
static int source_particle(const ctx_t* C, uint32_t h, part_t* p)
{
    const orc_problem* P = C->P;
    rng_t r;
    rng_init(&r, C->seed, h, 0u, 0u);
    const double u1 = rng_u(&r), u2 = rng_u(&r), u3 = rng_u(&r), u4 = rng_u(&r);
    double E = P->mono_E;
    if (P->n_bins > 0 && P->geometry != 2) {
        int b = 0;
        while (b < P->n_bins - 1 && !(C->cdf[b] > u1)) ++b;
        E = P->edges[b] + u2 * (P->edges[b + 1] - P->edges[b]);
    }
    double X[3] = {P->cx + (u3 - 0.5) * P->fx, P->cy + (u4 - 0.5) * P->fy, P->z_field};
    double d[3] = {0.0, 0.0, 1.0};
    double tS = -INFINITY; /* ray parameter of the source: parallel beams come from afar */
    if (P->geometry == 2) {
        /* phase-space record h mod n_psf; the particle moves forward only */
        const float* rec = P->psf + 8 * (size_t)(h % (uint32_t)P->n_psf);
        E = (double)rec[0];
        X[0] = (double)rec[1];
        X[1] = (double)rec[2];
        X[2] = (double)rec[3];
        const double a = (double)rec[4], b = (double)rec[5], c = (double)rec[6];
        const double nrm = sqrt(a * a + b * b + c * c);
        d[0] = a / nrm;
        d[1] = b / nrm;
        d[2] = c / nrm;
        tS = 0.0;
    } else if (P->geometry == 1) {
        const double a = X[0] - P->sx, b = X[1] - P->sy, c = X[2] - (P->z_field - P->ssd);
        const double nrm = sqrt(a * a + b * b + c * c);
        d[0] = a / nrm;
        d[1] = b / nrm;
        d[2] = c / nrm;
        tS = -nrm;
    }
    if (P->gantry_deg != 0.0) {
        /* rotation about the y axis through (iso_x, ., iso_z) */
        const double g = P->gantry_deg * PI / 180.0;
        const double cg = cos(g), sg = sin(g);
        const double px = X[0] - P->iso_x, pz = X[2] - P->iso_z;
        X[0] = P->iso_x + cg * px + sg * pz;
        X[2] = P->iso_z - sg * px + cg * pz;
        const double dx = d[0], dz = d[2];
        d[0] = cg * dx + sg * dz;
        d[2] = -sg * dx + cg * dz;
    }
    /* the particle enters where the ray from the source first meets the box
     * (slab method); the field point itself may lie inside the phantom */
    double t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double L = (double)C->n[a] * C->h[a];
        if (d[a] != 0.0) {
            double ta = (0.0 - X[a]) / d[a], tb = (L - X[a]) / d[a];
            if (ta > tb) {
                const double s = ta;
                ta = tb;
                tb = s;
            }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        } else if (X[a] < 0.0 || X[a] >= L) {
            t0 = INFINITY;
        }
    }
    p->E = E;
    if (!(t0 < t1) || t1 <= tS) return 0;
    const double tt = t0 > tS ? t0 : tS;
    for (int a = 0; a < 3; ++a) {
        p->x[a] = X[a] + tt * d[a];
        p->d[a] = d[a];
        double fl = floor(p->x[a] / C->h[a]);
        if (fl < 0.0) fl = 0.0;
        if (fl > (double)(C->n[a] - 1)) fl = (double)(C->n[a] - 1);
        p->iv[a] = (int)fl;
    }
    p->type = P->particle == 0 ? PT_PHOTON : PT_ELECTRON;
    p->nmfp = -1.0;
    rng_init(&p->rng, C->seed, h, 0u, 1u); /* transport continues at block 1 */
    return 1;
}

static void run_history(const ctx_t* C, uint32_t h, stack_t* st, tally_t* t)
{
    part_t p;
    const int hit = source_particle(C, h, &p);
    t->c.E_incident += p.E;
    if (!hit) {
        t->c.E_escaped += p.E;
        t->c.src_miss++;
        return;
    }
    if (p.type != PT_PHOTON && C->P->kerma_mode) {
        deposit(t, lin(C, p.iv), p.E);
        return;
    }
    st->n = 0;
    stack_push(st, &p);
    while (st->n > 0) {
        part_t q = st->a[--st->n];
        if (q.type == PT_PHOTON) transport_photon(C, &q, st, t);
        else if (C->P->electron_mode == 1) transport_electron_fixed(C, &q, st, t);
        else transport_electron(C, &q, st, t);
    }
}

/* --- context -------------------------------------------------------------------- */
static int ctx_init(ctx_t* C, const orc_problem* P, uint32_t seed)
{
    memset(C, 0, sizeof *C);
    if (!P || P->nx <= 0 || P->ny <= 0 || P->nz <= 0 || P->n_mats <= 0 || !P->density || !P->mat)
        return -1;
    C->P = P;
    C->seed = seed;
    C->n[0] = P->nx;
    C->n[1] = P->ny;
    C->n[2] = P->nz;
    C->h[0] = P->dx;
    C->h[1] = P->dy;
    C->h[2] = P->dz;
    C->nvox = (size_t)P->nx * (size_t)P->ny * (size_t)P->nz;
    /* A step that reaches a voxel face within this distance is taken without
     * the hinge deflection, as in the boundary-crossing algorithm that comes
     * with the random hinge (Kawrakow 2000). Without it, steps that end just
     * short of a face shrink geometrically toward it. */
    C->skin = 1e-3 * fmin(P->dx, fmin(P->dy, P->dz));
    C->rho = (double*)malloc(C->nvox * sizeof(double));
    C->tab = (orc_mat_tables*)calloc((size_t)P->n_mats, sizeof(orc_mat_tables));
    C->Rabs = (double*)calloc((size_t)P->n_mats, sizeof(double));
    double* rmax = (double*)calloc((size_t)P->n_mats, sizeof(double));
    for (size_t v = 0; v < C->nvox; ++v) {
        if (P->mat[v] >= P->n_mats || !(P->density[v] > 0.0f)) {
            free(rmax);
            return -1;
        }
        C->rho[v] = (double)P->density[v];
        if (C->rho[v] > rmax[P->mat[v]]) rmax[P->mat[v]] = C->rho[v];
    }
    for (int m = 0; m < P->n_mats; ++m) {
        orc_build_material(&P->mats[m], P->Wcc, P->kc, &C->tab[m]);
        C->Rabs[m] = orc_table_lookup(C->tab[m].R, P->Eabs_e);
    }
    /* photon majorant: node-wise maximum of rho_max(m) * mu_tot(m) over the
     * materials present; its interpolant bounds every material's */
    for (int i = 0; i < ORC_NE; ++i) {
        double mx = 0.0;
        for (int m = 0; m < P->n_mats; ++m) {
            const double val = rmax[m] * C->tab[m].muTot[i];
            if (val > mx) mx = val;
        }
        C->muhat[i] = mx;
    }
    free(rmax);
    /* macro cells: the smallest power-of-two side that leaves at most 4096 */
    C->cshift = 0;
    for (;;) {
        size_t nc = 1;
        for (int a = 0; a < 3; ++a) {
            C->cn[a] = (C->n[a] + (1 << C->cshift) - 1) >> C->cshift;
            nc *= (size_t)C->cn[a];
        }
        if (nc <= 4096) break;
        C->cshift += 1;
    }
    C->cellq = (unsigned char*)calloc((size_t)C->cn[0] * C->cn[1] * C->cn[2], 1);
    if (P->photon_mode == 1) {
        /* r_m: the largest ratio of material m's attenuation to the majorant
         * over the energy nodes; a voxel of density rho needs the scale
         * rho * r_m, and its cell takes the largest, rounded up to 255ths */
        double* r = (double*)calloc((size_t)P->n_mats, sizeof(double));
        for (int m = 0; m < P->n_mats; ++m)
            for (int i = 0; i < ORC_NE; ++i) {
                const double q = C->tab[m].muTot[i] / C->muhat[i];
                if (C->muhat[i] > 0.0 && q > r[m]) r[m] = q;
            }
        for (int z = 0; z < C->n[2]; ++z)
            for (int y = 0; y < C->n[1]; ++y)
                for (int x = 0; x < C->n[0]; ++x) {
                    const int iv[3] = {x, y, z};
                    const size_t v = lin(C, iv);
                    double qd = ceil(255.0 * (C->rho[v] * r[P->mat[v]]));
                    if (qd < 1.0) qd = 1.0;
                    if (qd > 255.0) qd = 255.0;
                    const size_t c = (size_t)(x >> C->cshift) +
                                     (size_t)C->cn[0] * ((size_t)(y >> C->cshift) +
                                                         (size_t)C->cn[1] * (size_t)(z >> C->cshift));
                    if ((unsigned char)qd > C->cellq[c]) C->cellq[c] = (unsigned char)qd;
                }
        free(r);
    }
    orc_build_ms_table(C->log2A);
    if (P->n_bins > 0) {
        C->cdf = (double*)malloc((size_t)P->n_bins * sizeof(double));
        double s = 0.0;
        for (int b = 0; b < P->n_bins; ++b) {
            s += P->weights[b];
            C->cdf[b] = s;
        }
        for (int b = 0; b < P->n_bins; ++b) C->cdf[b] = C->cdf[b] / s;
    }
    return 0;
}

static void ctx_free(ctx_t* C)
{
    free(C->rho);
    free(C->tab);
    free(C->Rabs);
    free(C->cdf);
    free(C->cellq);
}

static void counters_add(orc_counters* a, const orc_counters* b)
{
    a->ph_flights += b->ph_flights;
    a->ph_fictitious += b->ph_fictitious;
    a->ph_compton += b->ph_compton;
    a->ph_photo += b->ph_photo;
    a->ph_pair += b->ph_pair;
    a->ph_cutoff += b->ph_cutoff;
    a->ph_escaped += b->ph_escaped;
    a->el_steps += b->el_steps;
    a->el_hard_cand += b->el_hard_cand;
    a->el_hard_fict += b->el_hard_fict;
    a->el_moller += b->el_moller;
    a->el_brems += b->el_brems;
    a->el_absorbed += b->el_absorbed;
    a->el_escaped += b->el_escaped;
    a->el_boundary += b->el_boundary;
    a->el_hinge_trunc += b->el_hinge_trunc;
    a->pos_annihil += b->pos_annihil;
    a->push_ph += b->push_ph;
    a->push_el += b->push_el;
    a->src_miss += b->src_miss;
    a->E_incident += b->E_incident;
    a->E_deposited += b->E_deposited;
    a->E_escaped += b->E_escaped;
    a->E_pair_rest += b->E_pair_rest;
    a->E_annih_rest += b->E_annih_rest;
    a->watchdog += b->watchdog;
}

int orc_run(const orc_problem* P, uint64_t N, uint32_t seed, uint32_t h0, int nthreads,
            double* dose, double* dose2, orc_counters* out)
{
    if (N == 0 || P->n_batches <= 0 || !dose || !dose2 || !out) return -1;
    if ((uint64_t)h0 + N > 4294967296ull) return -1;
    ctx_t C;
    if (ctx_init(&C, P, seed) != 0) {
        ctx_free(&C);
        return -1;
    }
    const int B = P->n_batches;
    const int nt = nthreads > 0 ? nthreads : 1;
    const double V = P->dx * P->dy * P->dz;
    double** grids = (double**)calloc((size_t)nt, sizeof(double*));
    orc_counters* tc = (orc_counters*)calloc((size_t)nt, sizeof(orc_counters));
    double* Eb = (double*)malloc(C.nvox * sizeof(double));
    for (int k = 0; k < nt; ++k) grids[k] = (double*)malloc(C.nvox * sizeof(double));
    memset(dose, 0, C.nvox * sizeof(double));
    memset(dose2, 0, C.nvox * sizeof(double));
    memset(out, 0, sizeof *out);

    for (int b = 0; b < B; ++b) {
        /* batch b holds the relative indices i with floor(i*B/N) == b */
        const uint64_t i0 = ((uint64_t)b * N + (uint64_t)B - 1) / (uint64_t)B;
        const uint64_t i1 = ((uint64_t)(b + 1) * N + (uint64_t)B - 1) / (uint64_t)B;
        const uint64_t Nb = i1 - i0;
        if (Nb == 0) continue;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
        for (int k = 0; k < nt; ++k) {
            tally_t t;
            t.grid = grids[k];
            memset(t.grid, 0, C.nvox * sizeof(double));
            memset(&t.c, 0, sizeof t.c);
            stack_t st = {NULL, 0, 0};
            const uint64_t a0 = i0 + (uint64_t)k * Nb / (uint64_t)nt;
            const uint64_t a1 = i0 + (uint64_t)(k + 1) * Nb / (uint64_t)nt;
            for (uint64_t i = a0; i < a1; ++i) run_history(&C, (uint32_t)(h0 + i), &st, &t);
            free(st.a);
            tc[k] = t.c;
        }
        /* fixed-order reduction over tasks */
        memcpy(Eb, grids[0], C.nvox * sizeof(double));
        for (int k = 1; k < nt; ++k)
            for (size_t v = 0; v < C.nvox; ++v) Eb[v] += grids[k][v];
        for (int k = 0; k < nt; ++k) counters_add(out, &tc[k]);
        for (size_t v = 0; v < C.nvox; ++v) {
            dose[v] += Eb[v] / (C.rho[v] * V * (double)N);
            const double db = Eb[v] / (C.rho[v] * V * (double)Nb);
            dose2[v] += db * db;
        }
    }
    for (int k = 0; k < nt; ++k) free(grids[k]);
    free(grids);
    free(tc);
    free(Eb);
    ctx_free(&C);
    return 0;
}

/* --- test entry points ------------------------------------------------------------ */

int orc_trace(const orc_problem* P, uint32_t seed, uint32_t h, double* out, uint32_t cap,
              uint32_t* n_out)
{
    ctx_t C;
    if (ctx_init(&C, P, seed) != 0) {
        ctx_free(&C);
        return -1;
    }
    tally_t t;
    t.grid = (double*)calloc(C.nvox, sizeof(double));
    memset(&t.c, 0, sizeof t.c);
    stack_t st = {NULL, 0, 0};
    g_trace = out;
    g_trace_cap = cap;
    g_trace_n = 0;
    run_history(&C, h, &st, &t);
    *n_out = g_trace_n < cap ? g_trace_n : cap;
    g_trace = NULL;
    free(st.a);
    free(t.grid);
    ctx_free(&C);
    return 0;
}

int orc_first_interaction(const orc_problem* P, uint32_t seed, uint32_t h0, uint32_t n,
                          double* pos, int* type, uint64_t* n_fict)
{
    ctx_t C;
    if (ctx_init(&C, P, seed) != 0) {
        ctx_free(&C);
        return -1;
    }
    tally_t t;
    t.grid = (double*)calloc(C.nvox, sizeof(double));
    memset(&t.c, 0, sizeof t.c);
    for (uint32_t k = 0; k < n; ++k) {
        part_t p;
        type[k] = 0;
        pos[3 * k] = pos[3 * k + 1] = pos[3 * k + 2] = NAN;
        if (!source_particle(&C, h0 + k, &p)) continue;
        size_t v;
        int i;
        double f;
        const int real = P->photon_mode == 1 ? woodcock_cells(&C, &p, &t, &v, &i, &f)
                                             : woodcock(&C, &p, &t, &v, &i, &f);
        if (real) type[k] = select_type(&C, &p, v, i, f);
        for (int a = 0; a < 3; ++a) pos[3 * k + a] = p.x[a];
    }
    *n_fict = t.c.ph_fictitious;
    free(t.grid);
    ctx_free(&C);
    return 0;
}

void orc_sample_source(const orc_problem* P, uint32_t seed, uint32_t h0, uint32_t n, double* E,
                       double* x, double* d)
{
    ctx_t C;
    if (ctx_init(&C, P, seed) != 0) {
        ctx_free(&C);
        return;
    }
    for (uint32_t k = 0; k < n; ++k) {
        part_t p;
        const int hit = source_particle(&C, h0 + k, &p);
        E[k] = hit ? p.E : 0.0;
        for (int a = 0; a < 3; ++a) {
            x[3 * k + a] = hit ? p.x[a] : NAN;
            d[3 * k + a] = hit ? p.d[a] : NAN;
        }
    }
    ctx_free(&C);
}

void orc_sample_compton(double E, uint32_t seed, uint32_t n, double* eps, double* cost,
                        uint32_t* words)
{
    for (uint32_t k = 0; k < n; ++k) {
        rng_t r;
        rng_init(&r, seed, k, 0u, 0u);
        double t;
        eps[k] = sample_compton_eps(&r, E / MC2, &t);
        cost[k] = 1.0 - t;
        words[k] = 4u * (r.n - 1u) + (uint32_t)r.nw;
    }
}

void orc_sample_moller(double T, double Wcc, uint32_t seed, uint32_t n, double* eps)
{
    for (uint32_t k = 0; k < n; ++k) {
        rng_t r;
        rng_init(&r, seed, k, 0u, 0u);
        eps[k] = sample_moller_eps(&r, T, Wcc);
    }
}

void orc_sample_brems(double T, double kc, uint32_t seed, uint32_t n, double* k)
{
    for (uint32_t j = 0; j < n; ++j) {
        rng_t r;
        rng_init(&r, seed, j, 0u, 0u);
        k[j] = sample_brems_k(&r, T, kc);
    }
}

void orc_sample_ms(const double* log2A, double x, uint32_t seed, uint32_t n, double* omc)
{
    const double A = orc_ms_screening(log2A, x);
    for (uint32_t k = 0; k < n; ++k) {
        rng_t r;
        rng_init(&r, seed, k, 0u, 0u);
        omc[k] = sample_ms(&r, A);
    }
}

/* Electron step records of histories h0 .. h0+n-1: history k gets up to cap
 * records at out + 12*cap*k and n_out[k] is the number it made (see
 * orc_trace). Single-threaded. */
int orc_trace_range(const orc_problem* P, uint32_t seed, uint32_t h0, uint32_t n, double* out,
                    uint32_t cap, uint32_t* n_out)
{
    ctx_t C;
    if (ctx_init(&C, P, seed) != 0) {
        ctx_free(&C);
        return -1;
    }
    tally_t t;
    t.grid = (double*)calloc(C.nvox, sizeof(double));
    memset(&t.c, 0, sizeof t.c);
    stack_t st = {NULL, 0, 0};
    for (uint32_t k = 0; k < n; ++k) {
        g_trace = out + 12 * (size_t)cap * k;
        g_trace_cap = cap;
        g_trace_n = 0;
        run_history(&C, h0 + k, &st, &t);
        n_out[k] = g_trace_n < cap ? g_trace_n : cap;
    }
    g_trace = NULL;
    free(st.a);
    free(t.grid);
    ctx_free(&C);
    return 0;
}

/* For each source electron of histories h0 .. h0+n-1 (voxel-limited steps),
 * the first accepted hard-event candidate: the mass path travelled before it
 * (g/cm^2), the kinetic energy at it (the end of the step, before the event)
 * and its kind (1 Moller, 2 bremsstrahlung; 0 when the electron was absorbed
 * or escaped first, tau then being its whole mass path). Single-threaded. */
int orc_first_hard(const orc_problem* P, uint32_t seed, uint32_t h0, uint32_t n, double* tau,
                   double* T, int* kind)
{
    if (P->particle != 1 || P->electron_mode != 0 || P->kerma_mode) return -1;
    ctx_t C;
    if (ctx_init(&C, P, seed) != 0) {
        ctx_free(&C);
        return -1;
    }
    tally_t t;
    t.grid = (double*)calloc(C.nvox, sizeof(double));
    memset(&t.c, 0, sizeof t.c);
    stack_t st = {NULL, 0, 0};
    for (uint32_t k = 0; k < n; ++k) {
        part_t p;
        tau[k] = -1.0;
        T[k] = 0.0;
        kind[k] = 0;
        if (!source_particle(&C, h0 + k, &p)) continue;
        memset(&g_first, 0, sizeof g_first);
        g_first.active = 1;
        st.n = 0;
        transport_electron(&C, &p, &st, &t);
        tau[k] = g_first.tau;
        if (g_first.done) {
            T[k] = g_first.T;
            kind[k] = g_first.kind;
        }
    }
    memset(&g_first, 0, sizeof g_first);
    free(st.a);
    free(t.grid);
    ctx_free(&C);
    return 0;
}

/* One interaction of the transport code above, sample k drawn from stream
 * (seed, h = k, id 0) from block 0, on a particle with energy args[0] and
 * unit direction args[1..3] in voxel (0, 0, 0) of the problem's phantom (the
 * problem's Wcc, kc, E_abs and KERMA mode apply; E_abs = 0 keeps every
 * product). Record of ORC_SAMPLE_WORDS doubles per sample:
 *   [0] the particle's energy after the event, [1..3] its direction,
 *   [4] products made, [5..8] and [9..12] product E, u, v, w,
 *   [13], [14] product types (0 photon, 1 electron, 2 positron),
 *   [15] the sampled variable: Compton E'/E, Moller W/T, bremsstrahlung k,
 *        multiple scattering 1 - cos(theta) (args[4] = s/lambda_1 of the
 *        step), pair T-/(E - 2 mc^2).
 * which: ORC_EV_COMPTON, _MOLLER, _BREMS, _MS, _ANNIHILATION, _PAIR; for
 * ORC_EV_SOURCE the source of the problem makes history k's particle:
 * [0] its energy (0 for a miss), [1..3] direction, [5..7] entry point,
 * [15] 1 if it entered the phantom. words[k]: the stream words used. */
int orc_sample_event(const orc_problem* P, int which, const double* args, uint32_t seed,
                     uint32_t n, double* out, uint32_t* words)
{
    ctx_t C;
    if (which < ORC_EV_COMPTON || which > ORC_EV_SOURCE) return -1;
    if (ctx_init(&C, P, seed) != 0) {
        ctx_free(&C);
        return -1;
    }
    tally_t t;
    t.grid = (double*)calloc(C.nvox, sizeof(double));
    memset(&t.c, 0, sizeof t.c);
    stack_t st = {NULL, 0, 0};
    for (uint32_t k = 0; k < n; ++k) {
        double* r = out + (size_t)ORC_SAMPLE_WORDS * k;
        memset(r, 0, ORC_SAMPLE_WORDS * sizeof(double));
        part_t p;
        memset(&p, 0, sizeof p);
        if (which == ORC_EV_SOURCE) {
            const int hit = source_particle(&C, k, &p);
            r[0] = hit ? p.E : 0.0;
            for (int a = 0; a < 3; ++a) {
                r[1 + a] = hit ? p.d[a] : 0.0;
                r[5 + a] = hit ? p.x[a] : 0.0;
            }
            r[15] = hit;
            /* the source draws block 0 only; transport continues at block 1 */
            words[k] = 4u;
            continue;
        }
        p.type = which == ORC_EV_MOLLER || which == ORC_EV_MS ? PT_ELECTRON
               : which == ORC_EV_BREMS                       ? PT_ELECTRON
               : which == ORC_EV_ANNIHILATION                ? PT_POSITRON
                                                             : PT_PHOTON;
        p.E = args[0];
        for (int a = 0; a < 3; ++a) {
            p.d[a] = args[1 + a];
            p.x[a] = 0.5 * C.h[a];
            p.iv[a] = 0;
        }
        p.nmfp = -1.0;
        rng_init(&p.rng, seed, k, 0u, 0u);
        st.n = 0;
        const double E0 = p.E;
        double v = 0.0;
        switch (which) {
        case ORC_EV_COMPTON:
            compton(&C, &p, &st, &t);
            v = p.E / E0;
            break;
        case ORC_EV_MOLLER:
            moller(&C, &p, &st, &t);
            v = st.n ? st.a[0].E / E0 : (E0 - p.E) / E0;
            break;
        case ORC_EV_BREMS:
            brems(&C, &p, &st, &t);
            v = E0 - p.E;
            break;
        case ORC_EV_MS:
            v = ms_deflect(&p.rng, orc_ms_screening(C.log2A, args[4]), p.d);
            break;
        case ORC_EV_ANNIHILATION:
            annihilate(&C, &st, &t, &p.rng, p.x, p.iv);
            p.E = 0.0;
            break;
        case ORC_EV_PAIR:
            pair(&C, &p, &st, &t);
            v = st.n ? st.a[0].E / (E0 - 2.0 * MC2) : 0.0;
            p.E = 0.0;
            break;
        }
        r[0] = p.E;
        for (int a = 0; a < 3; ++a) r[1 + a] = p.d[a];
        r[4] = (double)st.n;
        for (size_t j = 0; j < st.n && j < 2; ++j) {
            r[5 + 4 * j] = st.a[j].E;
            for (int a = 0; a < 3; ++a) r[6 + 4 * j + a] = st.a[j].d[a];
            r[13 + j] = st.a[j].type;
        }
        r[15] = v;
        words[k] = 4u * (p.rng.n - (p.rng.n > 0 ? 1u : 0u)) + (p.rng.n > 0 ? (uint32_t)p.rng.nw : 0u);
    }
    free(st.a);
    free(t.grid);
    ctx_free(&C);
    return 0;
}
