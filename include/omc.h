/*
 * omc.h -- C ABI of the MI355X (gfx950) coupled photon-electron Monte Carlo dose
 * engine. The method is that of Tian et al., "An OpenCL-based Monte Carlo dose
 * calculation engine (oclMC) for coupled photon-electron transport"
 * (arXiv 1503.01722).
 *
 * Conventions for every entry point:
 *  - The return value is a status: OMC_OK (0) or a negative OMC_E* code. Nothing
 *    aborts or throws across this boundary. On error the context is unchanged
 *    (except for its last-error string) unless stated otherwise.
 *  - Host arrays passed in are copied during the call; the caller keeps
 *    ownership and may free them afterwards.
 *  - Host output arrays are allocated by the caller. Device output pointers are
 *    caller-owned device memory (for example a torch tensor's data_ptr()) valid
 *    on the stream given to the call.
 *  - A context is bound to the device current at omc_create and is not
 *    thread-safe: one thread at a time per context.
 *  - Units: MeV, cm, g/cm^3. Dose is MeV/g per source history (Sec. 2.2
 *    "Materials" of the paper reports dose in MeV/g per source particle).
 *  - Phantom arrays are nx*ny*nz values with x fastest, then y, then z.
 */
#ifndef OMC_H
#define OMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    OMC_OK = 0,
    OMC_EINVAL = -1,   /* invalid argument (sizes, NaN or non-positive density, ...) */
    OMC_ENOMEM = -2,   /* device or host allocation failed */
    OMC_EDEVICE = -3,  /* HIP runtime error or no device */
    OMC_ESTATE = -4,   /* call out of order (e.g. omc_run before omc_set_source) */
    OMC_EQUEUE = -5,   /* a secondary-particle queue overflowed; raise queue_factor */
    OMC_ENUMERIC = -6, /* non-finite result or energy ledger violated */
    OMC_EUNSUP = -7    /* unsupported configuration (e.g. too many materials) */
};

#define OMC_MAX_MATERIALS 32
#define OMC_MAX_DIM 1024
#define OMC_MAX_BATCHES 64
#define OMC_NE 512      /* energy nodes, uniform in log2 E over [0.01, 20] MeV */
#define OMC_NA 512      /* multiple-scattering screening table nodes */
#define OMC_TABLE_ROWS 11

typedef struct omc_ctx omc_ctx;

/* A material as an element composition (Sec. 2.1: the physics data of each
 * material are generated from a user-defined composition). */
typedef struct {
    int n_elem;
    const int* Z;            /* atomic numbers, n_elem */
    const double* A;         /* atomic weights g/mol, n_elem */
    const double* w_mass;    /* mass fractions, n_elem (normalised by the caller) */
    double I_eV;             /* mean excitation energy */
    double rho_nominal;      /* density used for the density-effect correction */
} omc_material;

/* Source (Sec. 2.2 "Materials": point source, SSD 100 cm, field defined at the
 * phantom surface, 6 MV spectrum or 15 MeV electrons). A field point is drawn
 * uniformly on an fx x fy rectangle centred at (cx, cy) in the plane z = z_field
 * of the gantry-0 frame; a point source sits at (sx, sy, z_field - ssd). The
 * frame is then rotated by gantry_deg about the y axis through (iso_x, iso_z),
 * and the particle enters where the ray from the source first meets the box.
 *
 * Phase space (geometry 2; the paper's source interface, Sec. 2.2 "Materials"):
 * history h takes record h mod n_psf of psf, n_psf x 8 floats per record:
 * energy (MeV, in (0, 20)), position x, y, z (cm) and direction u, v, w (any
 * non-zero length; normalised by the library) in the gantry-0 frame, and an
 * unused eighth float. The gantry rotation applies; the particle moves forward
 * from its recorded point to where it first meets the box (a record inside the
 * phantom starts where it is; one whose forward ray misses the box is an
 * escaped history). Spectrum and field members are ignored.
 *
 * The records are host memory (psf_on_device = 0), checked and copied by
 * omc_set_source and omc_run_beamlets, or device memory (psf_on_device = 1):
 * particles a caller's own GPU code wrote (the paper's user source function),
 * read in place. Device records must lie inside one HIP allocation of the
 * context's device, be complete when the call starts (the check runs on the
 * null stream) and stay allocated and unchanged until the next omc_set_source
 * (or, for beamlets, until omc_run_beamlets returns); the library checks them
 * on the device with the same conditions as host records, and a pointer
 * outside a device allocation, or an allocation too small for n_psf records,
 * is rejected with OMC_EINVAL before any kernel reads it. */
typedef struct {
    int particle;            /* 0 photon, 1 electron */
    int n_bins;              /* spectrum bins; 0 = mono-energetic mono_E */
    const double* edges;     /* n_bins + 1 bin edges, MeV, increasing */
    const double* weights;   /* n_bins non-negative weights (need not be normalised) */
    double mono_E;           /* MeV, used when n_bins == 0 */
    int geometry;            /* 0 parallel beam along the axis, 1 point source, 2 phase space */
    double ssd;              /* point source to field plane distance, cm */
    double z_field;          /* field plane z in the gantry-0 frame, cm */
    double fx, fy;           /* field size on the field plane, cm */
    double cx, cy;           /* field centre, cm */
    double sx, sy;           /* focal spot x, y (point source), cm */
    double gantry_deg;       /* rotation about y; 0 = beam along +z */
    double iso_x, iso_z;     /* rotation axis position, cm */
    int n_psf;               /* phase-space records (geometry 2), 1 .. 2^26 */
    const float* psf;        /* n_psf x 8 floats (geometry 2) */
    int psf_on_device;       /* 0: psf is host memory (copied); 1: device memory (read in place) */
} omc_source;

/* Transport parameters (Sec. 2.1 step limits; Sec. 2.2 "Materials" cut-offs)
 * and launch shape. Fill with omc_default_params() and override. */
typedef struct {
    double Eabs_e;           /* electron/positron absorption energy, MeV (0.2) */
    double Eabs_g;           /* photon absorption energy, MeV (0.05) */
    double Wcc;              /* Moller hard-event threshold, MeV (0.05) */
    double kc;               /* bremsstrahlung hard-event threshold, MeV (0.2) */
    double dmax_s;           /* maximum electron step, cm (0.5) */
    double f_E;              /* maximum fractional energy loss per step (0.25) */
    int n_batches;           /* batches for the uncertainty estimate (10) */
    int parity_fp64;         /* 1: transport in FP64 (bit-level parity build) */
    int kerma_mode;          /* 1: e-/e+ deposited where created */
    int csda_mode;           /* 1: no hinge, no multiple scattering, no hard events */
    int block_size;          /* work-items per work-group (256); multiple of 64 */
    int blocks_per_cu;       /* resident work-groups per CU for the transport grid (4) */
    int chunk_histories;     /* histories per source chunk (0 = min(n, 2^24)) */
    int queue_factor;        /* secondary queue capacity per source history (6) */
    int timing;              /* 1: record per-kernel HIP event times */
    int graph_depth;         /* 0: each photon+electron generation is launched from the host,
                                which reads the queue counts back after it; K in 1..64: the
                                launches of a run are captured once in a HIP graph, K
                                generations per source chunk, and replayed by later runs of
                                the same shape; particles still queued after a chunk's K
                                generations carry over into the next chunk's, and those left
                                after the last chunk are drained from the host (0) */
    int beamlet_group;       /* beamlets tallied together by omc_run_beamlets; 0 = as many as
                                half of the free device memory holds (0) */
    double sparse_threshold; /* omc_run_beamlets keeps a voxel when its dose exceeds this
                                fraction of the beamlet's largest voxel dose; 0 = every voxel
                                with a positive FP32 dose (0) */
    int straggler_lanes;     /* in a generation of more than 4 records per lane, a wave whose
                                input is used up and that has at most this many live lanes
                                left moves them, unchanged, to the next generation of their
                                type, where they run packed into full waves; 0 = off (16) */
    int electron_mode;       /* 0: Class II steps limited to one voxel (Sec. 2.1); 1: fixed
                                steps across voxels, the gDPM scheme Sec. 4 compares with: a
                                step is planned in mass thickness with the mass tables of the
                                material where it starts (they stand for every material it
                                crosses, density scaling only), limited by dmax_s at unit
                                density, f_E, E_abs and the hard-event mean free path, and
                                each voxel on its path receives the CSDA loss inside it (0) */
    int table_mode;          /* where the transport kernels read the per-material tables of
                                the materials present in the phantom: 1 in LDS, staged per
                                work-group (Sec. 2.2.2 keeps them in image memory; fails with
                                OMC_EUNSUP when they exceed a work-group's LDS); 2 in global
                                memory, through L2; 0 LDS while two work-groups still fit a
                                CU with them, else global (0). Results do not depend on it */
    int photon_mode;         /* 0: Woodcock flights with the phantom's majorant (Sec. 2.1);
                                1: with a majorant per macro cell, the remedy for the many
                                fictitious interactions Sec. 3.2 reports in heterogeneous
                                phantoms: cells of 2^k voxels per side (the smallest k that
                                leaves at most 4096 cells), each with the largest over its
                                voxels of rho times the material's largest ratio to the
                                majorant over the energy nodes, rounded up to 255ths; a
                                flight spends its optical depth -ln u cell by cell, and a
                                candidate is accepted with rho mu / mu_cell (0) */
    int tally_copies;        /* private copies of each batch's FP64 dose grid in a plain run
                                (1, 2, 4, 8 or 16): history h and its secondaries add their
                                deposits (Sec. 2.2.2: atomic additions to the dose counter)
                                into copy h mod tally_copies, and the fold sums the copies
                                before the batch statistics. Spreads the atomics on the few
                                hot voxels of a narrow beam over as many addresses; costs
                                tally_copies x the grid memory. Batched beamlets keep one
                                copy. Results do not depend on it (1) */
    int source_order;        /* 0: a source chunk's particles enter the photon or electron
                                queue in history order; 1: in descending energy groups
                                (quarter octaves), the paper's simulation of the source
                                energy bin by energy bin (Sec. 2.2.1, Table 1) without a
                                drain between bins: waves running together carry particles
                                of similar energy, the long-lived high-energy ones first.
                                Applies to spectra and phase spaces. Each particle's
                                transport depends on its own stream only, so counters are
                                unchanged and the dose only sums in another order (0) */
    int event_lanes;         /* an electron step that ends in a hard-event candidate (Sec.
                                2.1) leaves its lane waiting; the Moller/bremsstrahlung
                                sampling runs for the waiting lanes of a wave together once
                                this many wait (1..64) or no lane has a step left. Fewer:
                                passes with fewer lanes; more: more lanes idle meanwhile.
                                Results do not depend on it (12) */
} omc_params;

/* Per-run event counters and the energy ledger (all from the last run). */
typedef struct {
    uint64_t ph_flights, ph_fictitious, ph_compton, ph_photo, ph_pair, ph_cutoff, ph_escaped;
    uint64_t el_steps, el_hard_cand, el_hard_fict, el_moller, el_brems, el_absorbed, el_escaped;
    uint64_t el_boundary, el_hinge_trunc, pos_annihil, push_ph, push_el, src_miss;
    uint64_t watchdog;   /* particles stopped by the per-particle step bound (2^20) */
    double E_incident, E_deposited, E_escaped, E_pair_rest, E_annih_rest;
    uint64_t queue_hwm_ph, queue_hwm_el; /* largest queue occupancy seen */
    uint32_t iterations;                 /* photon/electron generations launched */
    uint32_t max_steps;                  /* most steps taken by one particle */
    uint64_t set_aside;                  /* particles moved to a later generation mid-track */
} omc_counters;

/* Per-kernel timing of the last run (params.timing == 1), HIP events on the
 * run's stream. HIP events cannot time the kernels of a graph, so with
 * graph_depth > 0 a timed run launches the same fixed-depth sequence without
 * capturing it. */
typedef struct {
    uint32_t launches[4];    /* 0 source, 1 photon, 2 electron, 3 fold or compaction */
    double total_ms[4];
    double run_ms;           /* whole run, first launch to last */
    int tables_global;       /* 1: the per-material tables were read from global memory
                                (params.table_mode), 0: staged in LDS; set by every run */
} omc_timing;

void omc_default_params(omc_params* p);

/* Create a context on the current HIP device for a voxelised phantom (Sec.
 * 2.1: each voxel has a density and a material). density: g/cm^3, finite and
 * > 0; material: ids < n_mats; mats: the material library, n_mats
 * compositions (1 <= n_mats <= OMC_MAX_MATERIALS; Sec. 2.1 supports 16, built
 * from user-defined compositions), copied; mats == NULL with n_mats 0 or 3
 * selects the built-in library 0 water, 1 lung, 2 cortical bone (the
 * materials of the paper's slab phantoms, Sec. 2.2 "Materials"). Sizes:
 * 1 <= nx,ny,nz <= 1024, voxel sizes > 0. Builds the closed-form tables (Sec.
 * 2.1) and uploads the phantom; the device holds the tables of the materials
 * present in the phantom only. Errors: OMC_EINVAL for any invalid argument
 * (*out is then NULL), OMC_EDEVICE without a device, OMC_ENOMEM. */
int omc_create(omc_ctx** out, int nx, int ny, int nz, double dx, double dy, double dz,
               const float* density, const uint8_t* material, const omc_material* mats,
               int n_mats);

/* Replace the phantom's densities and material ids (same dimensions, voxel
 * sizes and materials; copied, validated as in omc_create). The physics
 * tables of the materials are kept; the photon majorant, which depends on
 * the largest density of each material, is rebuilt. */
int omc_set_phantom(omc_ctx* ctx, const float* density, const uint8_t* material);

/* CT to phantom (Sec. 2.1: each voxel's density and material obtained from the
 * patient's CT by a mapping method, Schneider et al. 2000). Density: piecewise
 * linear in HU through the calibration nodes, the end node's density outside
 * them; on the segment hu[k] <= h < hu[k+1] it is, in FP64 with one rounding
 * per operation, rho[k] + (h - hu[k]) * ((rho[k+1] - rho[k]) / (hu[k+1] -
 * hu[k])), then rounded once to FP32. Material: material[b] of the first bin b
 * with h < hu_upper[b], the last bin when there is none. */
#define OMC_MAX_CT_NODES 64
typedef struct {
    int n_nodes;             /* calibration nodes, 2 .. OMC_MAX_CT_NODES */
    const double* hu;        /* n_nodes HU values, finite, strictly increasing */
    const double* rho;       /* n_nodes densities, g/cm^3, in [1e-6, 100] */
    int n_bins;              /* material bins, 1 .. OMC_MAX_MATERIALS */
    const double* hu_upper;  /* n_bins upper bounds, increasing (the last is not read) */
    const int* material;     /* n_bins library ids, < n_mats */
} omc_ct_map;

/* Replace the phantom's densities and materials by the mapping of a CT volume
 * hu (int16 HU, nx * ny * nz values, x fastest), mapped on the device. hu is
 * host memory (hu_on_device = 0, copied) or device memory on the context's
 * device (1; read once during the call, which must lie inside one allocation
 * holding every value, else OMC_EINVAL before any kernel reads it). Map errors
 * give OMC_EINVAL with the context unchanged. Synchronous. */
int omc_set_phantom_ct(omc_ctx* ctx, const int16_t* hu, int hu_on_device, const omc_ct_map* map);

/* Copy the phantom as the device holds it into host arrays of nx * ny * nz
 * densities (g/cm^3) and material ids (library ids), x fastest. Synchronous. */
int omc_get_phantom(const omc_ctx* ctx, float* density, uint8_t* material);

/* Set the source (copied). Spectrum weights must have a positive sum. */
int omc_set_source(omc_ctx* ctx, const omc_source* src);

/* Set parameters (copied). Rebuilds the electron tables when Wcc or kc change. */
int omc_set_params(omc_ctx* ctx, const omc_params* p);

/* The phantom grid of a context: voxels per axis and voxel sizes in cm (the
 * voxelised phantom of Sec. 2.1). Any output pointer may be NULL. */
int omc_get_geometry(const omc_ctx* ctx, int* nx, int* ny, int* nz, double* dx, double* dy,
                     double* dz);

/* The context's current parameters (after omc_autotune, the tuned ones). */
int omc_get_params(const omc_ctx* ctx, omc_params* out);

/* Transport histories h0 .. h0+n-1 (Sec. 2.1: each source particle and all
 * its secondaries, photons and electrons coupled, to absorption or escape;
 * Sec. 2.2.1, Table 1: the whole source simulated) with streams keyed by
 * (seed, h), and write dose in MeV/g per source history (the unit of Sec. 2.2
 * "Materials") and dose2 = sum over the n_batches batches of the squared batch
 * dose, from which the per-voxel uncertainty sigma_D of Sec. 3.1 follows as
 * sqrt((dose2 / B - dose^2) / (B - 1)); both nx*ny*nz doubles in caller-owned
 * host memory. h0 + n <= 2^32. Blocks until done. Errors: OMC_EINVAL (NULL
 * output, n == 0, h0 + n > 2^32), OMC_ESTATE without a source, OMC_EQUEUE,
 * OMC_ENOMEM, OMC_EDEVICE; OMC_ENUMERIC when the energy ledger (incident +
 * annihilation rest energy - pair rest energy = deposited + escaped) is off by
 * more than 1e-9 relative (the dose is still written). */
int omc_run(omc_ctx* ctx, uint64_t n, uint32_t seed, uint32_t h0, double* dose,
            double* dose2);

/* As omc_run (Sec. 2.1 transport; dose and sigma_D as above), with dose and
 * dose2 in caller-owned device memory, launched on
 * hip_stream (a hipStream_t; NULL = default stream). Returns when the run is
 * complete on that stream. */
int omc_run_device(omc_ctx* ctx, uint64_t n, uint32_t seed, uint32_t h0, double* d_dose,
                   double* d_dose2, void* hip_stream);

/* For callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * omc_run_device without any device allocation. The run's queues, tally grids,
 * statistics, control words and source description live in the library's
 * fixed device scratch, a 128 MiB array that every GPU the library runs on
 * holds until the process ends; nothing else is allocated or freed.
 * Results equal omc_run_device's for the same inputs (same streams, same event
 * counters; dose to summation order). Limits: n_batches x tally_copies x nx*ny*nz <= 6291456
 * tally doubles (else OMC_EINVAL); the source description (beams and spectra)
 * within 1 MiB (else OMC_EINVAL); the queues hold about 50000 (FP32) or 27000
 * (FP64) source histories per chunk, which the call sizes itself. Preconditions:
 * the physics tables of the context's precision (and the phase-space copy of
 * a host-record source, and the cell scales for photon_mode 1) are already on
 * the device: run omc_run or omc_run_device once after omc_create, omc_set_params
 * or omc_set_source, else OMC_ESTATE. dose and dose2 must each lie inside one
 * device allocation of the context's device holding nx*ny*nz doubles (else
 * OMC_EINVAL). Every call on one GPU shares that GPU's scratch, which keeps
 * the last call's contents (each call clears what must start at zero): calls
 * that overlap on one GPU, from any context or thread, race and must not be
 * made. Launched on hip_stream (NULL = default stream) with host-driven
 * generations; returns when the run is complete on that stream. */
int omc_run_device_static(omc_ctx* ctx, uint64_t n, uint32_t seed, uint32_t h0,
                          double* d_dose, double* d_dose2, void* hip_stream);

/* One beamlet of a batched run: a source with its own history count and
 * history ids. (The paper transports one beam per run and tunes only the
 * number of work-items per launch, Sec. 2.2.2; batching many small beams into
 * one run keeps the device full where one beamlet alone cannot.) */
typedef struct {
    omc_source src;          /* geometry and spectrum; arrays read during the call */
    uint64_t n_histories;    /* >= 1 */
    uint32_t h0;             /* histories h0 .. h0+n-1, streams keyed by (seed, h); h0 + n <= 2^32 */
} omc_beamlet;

/* Per-beamlet dose in compressed sparse rows. Allocated by omc_run_beamlets,
 * released with omc_free_sparse. */
typedef struct {
    int n_beamlets;
    int on_device;           /* 1: voxel and dose are device memory of the context's device */
    uint64_t nnz;
    uint64_t* row_ptr;       /* host memory, n_beamlets + 1: beamlet b owns [row_ptr[b], row_ptr[b+1]) */
    uint32_t* voxel;         /* nnz linear voxel indices (x fastest), increasing within a row */
    float* dose;             /* nnz doses, MeV/g per history of that beamlet */
} omc_sparse_out;

/* Transport n_beamlets beams in one run per group of params.beamlet_group
 * beamlets: their histories are interleaved in the same source chunks and
 * particle generations (one launch sequence, a captured graph when
 * graph_depth > 0), each beamlet tallied in an FP64 grid of its own, and every
 * grid compacted on the device into the CSR rows of *out (FP32 dose, voxels
 * kept per sparse_threshold). The dose of a beamlet equals the dose omc_run
 * gives for its source, history count and h0 with the same seed (same streams,
 * same counters; summation order aside). All beamlets must have the same
 * particle type. on_device: 1 leaves voxel and dose in device memory (launched
 * on hip_stream, NULL = default stream), 0 copies them to host memory.
 * Counters and timing of the call are those of omc_get_counters/omc_get_timing.
 * Errors: OMC_EINVAL for a NULL or invalid beamlet (rules of omc_set_source,
 * n_histories >= 1, 1 <= n_beamlets <= 65535), OMC_EQUEUE, OMC_ENOMEM,
 * OMC_ENUMERIC as omc_run; *out is zeroed first and left empty on error. */
int omc_run_beamlets(omc_ctx* ctx, const omc_beamlet* beamlets, int n_beamlets, uint32_t seed,
                     int on_device, void* hip_stream, omc_sparse_out* out);

/* Release what omc_run_beamlets allocated in *out and zero it. NULL is ignored. */
void omc_free_sparse(omc_sparse_out* out);

/* Launch-shape autotuner (the paper sets its number of work-items M by hand,
 * Sec. 2.2.2). Times runs of n_probe histories of the current source with the
 * current physics parameters over work-group size, work-groups per CU, source
 * chunk size (up to 2^24 histories, or up to the whole probe while its queues
 * take at most half the free device memory) and graph depth, then
 * tally_copies 2, 4 and 8 on the fastest
 * shape (while the copies take at most a quarter of the free device memory),
 * event_lanes 8, 24 and 32 and, for a spectrum or phase-space source, the other
 * source_order; keeps
 * the fastest, sizes queue_factor from the
 * queue high-water marks it saw, and applies the result to ctx (as
 * omc_set_params would). *best receives it when best != NULL. Each candidate
 * runs three times (the first builds its graph). Errors: OMC_ESTATE without a
 * source, OMC_EINVAL for n_probe == 0 or > 2^31, run errors if no candidate
 * completes. */
int omc_autotune(omc_ctx* ctx, uint64_t n_probe, uint32_t seed, omc_params* best);

/* The event counters and energy ledger of the last run (the interactions of
 * Sec. 2.1 by type, the secondaries pushed onto the stacks of Sec. 2.2.1 and
 * the energies of the ledger), copied to *out. Errors: OMC_EINVAL for NULL. */
int omc_get_counters(const omc_ctx* ctx, omc_counters* out);
/* Per-kernel HIP-event times of the last run (see omc_timing; no passage of
 * the paper: measurement). Errors: OMC_EINVAL for NULL. */
int omc_get_timing(const omc_ctx* ctx, omc_timing* out);

/* Random numbers (Sec. 2.2.3 gives every work-item its own stream; here a
 * counter-based generator keyed by history instead of RANECU seeded per
 * work-item). Words of the Philox4x32-10 stream keyed by (seed, h) for particle id q,
 * blocks n0 .. n0+nblocks-1, computed on the GPU: out holds 4*nblocks words
 * (host memory, caller-owned). */
int omc_debug_philox(uint32_t seed, uint32_t h, uint64_t q, uint32_t n0, uint32_t nblocks,
                     uint32_t* out);

/* Debugging aid: transport history h alone (stream key (seed, h)) and record
 * every electron step: out receives up to max_records records of 12 doubles
 * {code, id_lo, id_hi, stream position, x, y, z, u, v, w, E, voxel} taken after
 * the step (code 16 + limiter + 8 * crossed, 64 = absorbed); *n_records gets
 * the number written. Records of one particle are in step order. */
int omc_debug_trace(omc_ctx* ctx, uint32_t seed, uint32_t h, double* out, uint32_t max_records,
                    uint32_t* n_records);

/* Test entry: run one interaction of the transport code on the GPU, n times,
 * for element-by-element comparison with a CPU implementation. Sample k draws
 * from stream (seed, h = k, particle id 0) from block 0 (Sec. 2.2.3 gives each
 * work-item its own random stream) and acts on a particle of energy args[0]
 * (MeV) and unit direction args[1..3] in voxel (0, 0, 0) of the context's
 * phantom, with the context's Wcc and kc and its precision (parity_fp64);
 * every product is kept (absorption energies and KERMA mode do not apply).
 * which (Sec. 2.1 physics):
 *   0 Compton scattering (Klein-Nishina), 1 Moller event, 2 bremsstrahlung
 *   event, 3 multiple-scattering deflection of a step with args[4] =
 *   s / lambda_1, 4 positron annihilation at rest, 5 pair production,
 *   6 the context's source (Sec. 2.2 "Materials"): history k's entering
 *   particle (args unused; omc_set_source first, else OMC_ESTATE).
 * out: n records of 16 doubles (host memory, caller-owned): [0] the
 * particle's energy after the event, [1..3] its direction, [4] products made,
 * [5..8] and [9..12] the first two products' energy and direction, [13] and
 * [14] their types (0 photon, 1 electron, 2 positron), [15] the sampled
 * variable: Compton E'/E, Moller W/T, bremsstrahlung k (MeV), 1 - cos(theta),
 * pair T-/(E - 2 mc^2). For the source: [0] energy (0 when the ray misses the
 * phantom), [1..3] direction, [5..7] entry point (cm), [15] 1 if it entered.
 * words: n stream words used (host memory). 1 <= n <= 2^22; E in (0, 20] MeV;
 * pair needs E > 2 mc^2; else OMC_EINVAL. Synchronous; allocates and frees
 * its own device scratch. */
int omc_debug_sample(omc_ctx* ctx, int which, const double* args, uint32_t seed, uint32_t n,
                     double* out, uint32_t* words);

/* Host-only (no device needed): the engine's own table builder. out receives
 * OMC_TABLE_ROWS x OMC_NE doubles in the row order muC, muPE, muPair, muTot,
 * Scol, Srad, R, sigM, sigB, sigHat, K1 (units cm^2/g, MeV cm^2/g, g/cm^2). */
int omc_host_tables(const omc_material* mat, double Wcc, double kc, double* out);
/* Host-only: log2 of the screening parameter A at OMC_NA nodes uniform in
 * log2(s/lambda_1) over [-24, 3]. */
int omc_host_ms_table(double* out);

/* Last error message of ctx (or of the calling thread when ctx is NULL). */
const char* omc_last_error(const omc_ctx* ctx);

/* Release the context and every device and host allocation it owns (no
 * passage of the paper: resource management). NULL is ignored. Sparse outputs
 * of omc_run_beamlets are the caller's and stay valid until omc_free_sparse. */
void omc_destroy(omc_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
