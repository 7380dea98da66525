/*
 * omc_oracle.h -- plain FP64 CPU oracle for coupled photon-electron Monte Carlo
 * dose calculation (Tian et al., "An OpenCL-based Monte Carlo dose calculation
 * engine (oclMC) for coupled photon-electron transport", arXiv 1503.01722).
 *
 * THIS IS TEST INFRASTRUCTURE. Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load or call it. The GPU product
 * path never links, imports or executes anything in this directory, and this
 * directory shares no code, header, table or constant generator with it.
 *
 * What it computes (section references are to the paper):
 *   - Sec. 2.1: voxelised phantom (density + material per voxel); analogue
 *     photon transport with Woodcock tracking, Compton (Klein-Nishina),
 *     photoelectric absorption and a rough pair model; Class II condensed
 *     history electrons (CSDA loss with restricted stopping power, random-hinge
 *     multiple scattering, Moller and bremsstrahlung hard events, positron
 *     annihilation at the end of the track).
 *   - Sec. 2.2 "Materials" (the second 2.2): cut-offs, point source, dose in
 *     MeV/g per source particle.
 *   - Sec. 3.1: per-voxel uncertainty (batch method).
 * Where the paper is silent the oracle follows the readings written down in
 * the design notes of the repository (grids, closed forms, stream layout).
 *
 * Everything is double precision and written step by step; nothing is blocked,
 * fused or reordered beyond what the algorithm states.
 *
 * Pins (tests under tests/): Philox against rocRAND's host-callable Philox;
 * closed forms against numerical quadrature, textbook limits and PDG/ESTAR
 * values; samplers by chi-square against analytic CDFs; Woodcock flights
 * against exp(-mu x); CSDA depth-dose against an independent range integral;
 * the first real hard event of an electron against the survival
 * exp(-integral sigma_hard) along its CSDA track; the mean direction cosine
 * along a track against the product of the per-step exp(-s/lambda_1) and the
 * first step's moments against the random hinge; momentum and energy balance
 * of Compton and Moller events, the bremsstrahlung angle, isotropic
 * annihilation; the energy ledger to 1e-9. Planted mistakes in a copy of the
 * transport code fail these pins. The photoelectric and pair cross sections are
 * rough models (the paper uses XCOM data, absent here): they are pinned only
 * by their scaling laws and order of magnitude ("parity partially pinned").
 */
#ifndef OMC_ORACLE_H
#define OMC_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NE 512   /* energy nodes, uniform in log2 E over [ORC_ELO, ORC_EHI] */
#define ORC_ELO 0.01 /* MeV */
#define ORC_EHI 20.0 /* MeV */
#define ORC_NA 512   /* multiple-scattering table nodes, uniform in log2 x */
#define ORC_XLO (-24.0) /* log2 of the smallest tabulated x = s/lambda_1 */
#define ORC_XHI 3.0     /* log2 of the largest tabulated x */

typedef struct {
    int n_elem;
    const int* Z;
    const double* A;      /* g/mol */
    const double* w;      /* mass fractions */
    double I_eV;          /* mean excitation energy */
    double rho_nom;       /* nominal density for the density effect, g/cm^3 */
} orc_material;

/* Per-material tables at the energy nodes E_i = 2^(log2 ELO + i*dL). */
typedef struct {
    double muC[ORC_NE], muPE[ORC_NE], muPair[ORC_NE], muTot[ORC_NE]; /* cm^2/g */
    double Scol[ORC_NE], Srad[ORC_NE]; /* restricted stopping powers, MeV cm^2/g */
    double R[ORC_NE];                   /* range from ELO, g/cm^2 */
    double sigM[ORC_NE], sigB[ORC_NE];  /* hard Moller / bremsstrahlung, cm^2/g */
    double sigHat[ORC_NE];              /* running max of sigM+sigB over nodes <= i */
    double K1[ORC_NE];                  /* 1/(rho lambda_1), cm^2/g */
} orc_mat_tables;

typedef struct {
    uint64_t ph_flights, ph_fictitious, ph_compton, ph_photo, ph_pair, ph_cutoff, ph_escaped;
    uint64_t el_steps, el_hard_cand, el_hard_fict, el_moller, el_brems, el_absorbed, el_escaped;
    uint64_t el_boundary, el_hinge_trunc, pos_annihil, push_ph, push_el, src_miss;
    double E_incident, E_deposited, E_escaped, E_pair_rest, E_annih_rest;
    uint64_t watchdog; /* walks stopped by a bound that exact arithmetic never reaches */
} orc_counters;

typedef struct {
    /* phantom: box [0,nx*dx) x [0,ny*dy) x [0,nz*dz), x fastest */
    int nx, ny, nz;
    double dx, dy, dz;
    const float* density;   /* g/cm^3 */
    const uint8_t* mat;
    int n_mats;
    const orc_material* mats;
    /* source */
    int particle;           /* 0 photon, 1 electron */
    int n_bins;             /* 0: mono_E */
    const double* edges;    /* n_bins+1 */
    const double* weights;  /* n_bins */
    double mono_E;
    int geometry;           /* 0 parallel, 1 point, 2 phase space */
    double ssd;             /* source to field plane along the axis */
    double z_field;         /* field plane z in the gantry-0 frame */
    double fx, fy, cx, cy;  /* field size and centre on the field plane */
    double sx, sy;          /* focal point x,y in the gantry-0 frame */
    double gantry_deg, iso_x, iso_z;
    /* parameters */
    double Eabs_e, Eabs_g, Wcc, kc, dmax_s, f_E;
    int n_batches;
    int kerma_mode;         /* e+- deposited where created */
    int csda_mode;          /* no hinge, no multiple scattering, no hard events */
    int electron_mode;      /* 0 voxel-limited steps (Sec. 2.1), 1 fixed steps across voxels (Sec. 4) */
    /* phase-space source (geometry 2): history h takes record h mod n_psf of
     * psf (8 floats: E, x, y, z, u, v, w, unused) */
    int n_psf;
    const float* psf;
    /* photon flights: 0 Woodcock with the phantom majorant (Sec. 2.1); 1 with
     * a majorant per macro cell (the cure for the fictitious interactions
     * Sec. 3.2 reports in heterogeneous phantoms), see woodcock_cells */
    int photon_mode;
} orc_problem;

/* --- random numbers (Philox4x32-10, Salmon et al. SC'11) ------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t x);
void orc_u01_array(const uint32_t* x, size_t n, double* out);
/* words of stream (seed, h, q) starting at block n0: 4*nblocks words */
void orc_stream_words(uint32_t seed, uint32_t h, uint64_t q, uint32_t n0, uint32_t nblocks,
                      uint32_t* out);

/* --- closed forms, per element (Z, A) or per electron ---------------------- */
double orc_sigma_kn(double E);                         /* cm^2 per electron */
double orc_sigma_pe_atom(int Z, double E);             /* cm^2 per atom */
double orc_sigma_pair_atom(int Z, double E);           /* cm^2 per atom */
double orc_inv_X0_element(int Z, double A);            /* cm^2/g */
double orc_material_inv_X0(const orc_material* m);
double orc_scol_restricted(const orc_material* m, double T, double Wcc); /* MeV cm^2/g */
double orc_srad_restricted(const orc_material* m, double T, double kc);
double orc_sigma_moller(const orc_material* m, double T, double Wcc);    /* cm^2/g */
double orc_sigma_brems(const orc_material* m, double T, double kc);      /* cm^2/g */
double orc_K1(const orc_material* m, double T);                          /* cm^2/g */
double orc_ms_m1(double A);                 /* mean of 1-cos for screening A */

/* --- tables ----------------------------------------------------------------- */
double orc_node_energy(int i);
int orc_build_material(const orc_material* m, double Wcc, double kc, orc_mat_tables* out);
void orc_build_ms_table(double* log2A /* ORC_NA */);
double orc_table_lookup(const double* y, double E);   /* lerp in log2 E */
double orc_range_inverse(const double* R, double Rv);  /* exact inverse of the lerp */
double orc_ms_screening(const double* log2A, double x);

/* --- samplers (each draws from stream (seed, h=i, q=0) from block 0) -------- */
/* Compton: out eps, cos(theta) and the number of words used, for n samples. */
void orc_sample_compton(double E, uint32_t seed, uint32_t n, double* eps, double* cost,
                        uint32_t* words);
void orc_sample_moller(double T, double Wcc, uint32_t seed, uint32_t n, double* eps);
void orc_sample_brems(double T, double kc, uint32_t seed, uint32_t n, double* k);
void orc_sample_ms(const double* log2A, double x, uint32_t seed, uint32_t n, double* one_minus_cos);
/* Rotate unit vector d by polar (cost, sint) and azimuth (cphi, sphi). */
void orc_rotate(double d[3], double cost, double sint, double cphi, double sphi);
/* Source: for histories h0..h0+n-1, the entering particle (E, x, d) or E=0 for a miss. */
void orc_sample_source(const orc_problem* p, uint32_t seed, uint32_t h0, uint32_t n,
                       double* E, double* x, double* d);

/* --- transport ---------------------------------------------------------------- */
/* Narrow-beam helper: each source photon is flown (Woodcock) until its first
 * real interaction; returns its position and type (1 Compton, 2 photo,
 * 3 pair, 0 escaped). Fictitious events are counted in *n_fict. */
int orc_first_interaction(const orc_problem* p, uint32_t seed, uint32_t h0, uint32_t n,
                          double* pos, int* type, uint64_t* n_fict);

/* Debugging aid: transport history h alone, recording 12 doubles per electron
 * step {code, id_lo, id_hi, stream position, x, y, z, u, v, w, E, voxel}
 * after the step (code 16 + limiter + 8 * crossed, 64 = absorbed). Not
 * thread-safe. */
int orc_trace(const orc_problem* p, uint32_t seed, uint32_t h, double* out, uint32_t cap,
              uint32_t* n_out);

/* Step records of histories h0 .. h0+n-1, cap records each (history k at
 * out + 12*cap*k, n_out[k] records). */
int orc_trace_range(const orc_problem* p, uint32_t seed, uint32_t h0, uint32_t n, double* out,
                    uint32_t cap, uint32_t* n_out);

/* First accepted hard-event candidate of each source electron (voxel-limited
 * steps): mass path before it (g/cm^2), energy at it, kind (1 Moller, 2
 * bremsstrahlung, 0 none before absorption or escape). */
int orc_first_hard(const orc_problem* p, uint32_t seed, uint32_t h0, uint32_t n, double* tau,
                   double* T, int* kind);

/* One interaction of the transport code per sample (see transport.c for the
 * record layout of ORC_SAMPLE_WORDS doubles). */
#define ORC_SAMPLE_WORDS 16
enum { ORC_EV_COMPTON = 0, ORC_EV_MOLLER, ORC_EV_BREMS, ORC_EV_MS, ORC_EV_ANNIHILATION,
       ORC_EV_PAIR, ORC_EV_SOURCE };
int orc_sample_event(const orc_problem* p, int which, const double* args, uint32_t seed,
                     uint32_t n, double* out, uint32_t* words);

/* Full run of histories h0..h0+N-1. dose, dose2: nx*ny*nz, MeV/g per history
 * and sum over batches of the squared batch dose. Returns 0 or <0 on error. */
int orc_run(const orc_problem* p, uint64_t N, uint32_t seed, uint32_t h0, int nthreads,
            double* dose, double* dose2, orc_counters* c);

#ifdef __cplusplus
}
#endif
#endif
