// engine.hpp -- data shared by the host runtime and the gfx950 kernels.
//
// Layout in HBM (all allocations made once per context, sized for the run):
//   phantom     rho f32[nvox], mat u8[nvox] (library ids)    x fastest
//               vox u32x2[nvox] {rho bits, table slot}       transport copy
//   tables      for the materials present in the phantom (slots, library
//               order): photon R4[n][NE] {mu_tot, mu_C, mu_PE, 0} (cm^2/g),
//               majorant R[NE] (1/cm), electron R2[n][NE] {K1, sigma_hat},
//               hard R2[n][NE] {sigma_M, sigma_B}, range R[n][NE] and its
//               u16 cell index [n][kRangeCells], ms log2 A R[NA], R(E_abs) R[n]
//   queues      four structure-of-arrays particle queues (photon cur/next,
//               electron cur/next), each {x,y,z,u,v,w,E} R, voxel u32 packed
//               (ix | iy<<10 | iz<<20), history u32, particle id 2 x u32,
//               tag u32 (type | resumed 0x80 | tally cell << 8), and for
//               particles set aside mid-track their stream position u32 and
//               one R of step state; a control block of {count, head} per queue
//   tally       f64[cells][copies][nvox] (the one FP64 step on the GPU): a
//               cell is a batch of a plain run or a beamlet of a batched-beamlet
//               run; a plain run may keep several private copies of each batch
//               (tally_copies), history h adding into copy h mod copies
//   sources     BeamSrc[n_beams], history prefix u64[n_beams + 1], spectra
//   counters    u64[kNumCounters] and f64 energies[kNumEnergies]
// R is float for production transport and double for the parity build.
#pragma once

#include <cstddef>
#include <cstdint>

namespace omc {

constexpr int kMaxMaterials = 32;  // materials of a context's library
constexpr int kMaxCtNodes = 64;    // HU -> density calibration nodes
constexpr int kMaxCtBins = 32;     // HU -> material bins

enum Counter : int {
    C_PH_FLIGHTS = 0,
    C_PH_FICT,
    C_PH_COMPTON,
    C_PH_PHOTO,
    C_PH_PAIR,
    C_PH_CUTOFF,
    C_PH_ESCAPED,
    C_EL_STEPS,
    C_EL_HARD_CAND,
    C_EL_HARD_FICT,
    C_EL_MOLLER,
    C_EL_BREMS,
    C_EL_ABSORBED,
    C_EL_ESCAPED,
    C_EL_BOUNDARY,
    C_EL_HINGE_TRUNC,
    C_POS_ANNIHIL,
    C_PUSH_PH,
    C_PUSH_EL,
    C_SRC_MISS,
    C_WATCHDOG,
    C_SET_ASIDE,
    kNumCounters
};

enum Energy : int { EN_INCIDENT = 0, EN_DEPOSITED, EN_ESCAPED, kNumEnergies };

enum PType : int { PT_PHOTON = 0, PT_ELECTRON = 1, PT_POSITRON = 2 };

constexpr uint32_t kResBlockSlots = 128;  // output slots a wave reserves per atomic
constexpr uint32_t kHoleTag = 0xFFFFFFFFu;  // queue slot reserved but never filled
constexpr int kTabNE = 512;
constexpr int kTabNA = 512;
constexpr int kRangeCells = 1024;  // range-inverse index cells per material

template <typename R>
struct QueueView {
    R *x, *y, *z, *u, *v, *w, *E;
    uint32_t* vox;
    uint32_t* hist;
    uint32_t* qlo;
    uint32_t* qhi;
    uint32_t* tag;    // type | resumed (0x80) | cell << 8; kHoleTag for a reserved, unfilled slot
    // state of a particle set aside mid-track (tag bit 0x80): stream position
    // in words, and the remaining hard-event mean free paths (electrons) or
    // the pending-Compton flag (photons)
    uint32_t* aux_pos;
    R* aux_f;
    uint32_t* count;  // number of records written (atomic append)
    uint32_t* head;   // next record to hand out (atomic take)
    uint32_t cap;
};

template <typename R>
struct PhantomView {
    const float* rho;
    const uint8_t* mat;
    int nx, ny, nz;
    R hx, hy, hz;
    R ihx, ihy, ihz;  // 1/h (production transport only)
    R fnx, fny, fnz;  // the dimensions in the transport precision
    // density bits and material id of each voxel side by side: the transport
    // kernels gather both with one 8-byte load (one cache line)
    const uint2* vox;
};

template <typename R>
struct TableView {
    const R* ph;      // [n_mats][NE][4]
    const R* muhat;   // [NE]
    const R* el;      // [n_mats][NE][2]: K1, sigma_hat (staged in LDS)
    const R* hard;    // [n_mats][NE][2]: sigma_M, sigma_B (global memory)
    const R* rtab;    // [n_mats][NE]: CSDA range R(E)
    const uint16_t* ridx;  // [n_mats][kRangeCells]: range node of each range cell
    const R* msA;     // [NA]
    const R* Rabs;    // [n_mats]
    int n_mats;
    R L0, DL, INV;    // energy grid
    // range cells: the FP32 bit pattern of R shifted right by rshift, minus
    // rbase, clamped to [0, rcells-1]; a monotone pseudo-logarithm of R
    uint32_t rshift, rbase, rcells;
    R XLO, XHI, XINV; // multiple-scattering grid
    R ELo, EHi;
};

template <typename R>
struct ParamView {
    R Eabs_e, Eabs_g, Wcc, kc, dmax_s, one_minus_fE;
    R skin;  // boundary skin depth: 1e-3 of the smallest voxel side
    int kerma, csda;
};

struct TallyView {
    double* grid;        // [cells][copies][nvox]: a particle adds into grid[cell * nvox + v]
    size_t nvox;
    uint32_t copy_mask;  // copies - 1 (copies a power of two); the source sets a
                         // history's cell to batch * copies + (h & copy_mask)
};

// Values that change from run to run, read by the kernels from device memory
// so that a captured launch sequence can be replayed for another run.
struct RunDesc {
    uint32_t seed;
    uint32_t n_batches;  // cells of a plain run
    uint64_t n_total;    // histories of the run
};

struct StatsView {
    unsigned long long* counters;  // [n_rows][kNumCounters], summed at the end of a run
    double* energies;              // [n_rows][kNumEnergies]
    uint32_t n_rows;
    uint32_t* overflow;            // set to 1 when a push found its queue full
    uint32_t* max_steps;           // longest particle (steps) of the run
    uint32_t* hwm;                 // [2] queue high-water marks in slots: electrons, photons
};

// One beam of a run: a plain run has one, a batched-beamlet run one per
// beamlet. Spectra of all beams are concatenated in SourceView::cdf / edges.
template <typename R>
struct BeamSrc {
    R mono_E;
    R ssd, z_field, fx, fy, cx, cy, sx, sy;
    R cg, sg, iso_x, iso_z;  // cos/sin of the gantry angle (host FP64)
    int n_bins;              // 0: mono-energetic
    int cdf_off, edge_off;   // first entry of this beam's cdf / edges
    int point;               // 1 point source
    int rotate;              // gantry != 0
    uint32_t h0;             // history id of the beam's first history
    int n_psf;               // phase space: records (history h takes h mod n_psf); 0 = analytic
    const float* psf;        // this beam's records, 8 floats each (device memory)
};

template <typename R>
struct SourceView {
    const BeamSrc<R>* beams;
    const uint64_t* first;  // [n_beams + 1] prefix sums of the beams' history counts
    const double* cdf;      // per beam n_bins, FP64 running sum normalised by its last entry
    const R* edges;         // per beam n_bins + 1
    int n_beams;
    int particle;           // 0 photon, 1 electron (all beams of a run)
    int cell_mode;          // 0: cell = batch of the history; 1: cell = beam index
};

// Step trace of one history (debugging aid): 12 doubles per electron step.
struct TraceView {
    double* buf;
    uint32_t* n;
    uint32_t cap;
    uint32_t h;
    int on;
};
constexpr int kTraceWords = 12;

// Macro cells of 2^shift voxels per side for the photon majorant per cell:
// q[cell] (cells x fastest, at most kMaxCells) is the cell's majorant scale
// in 255ths of the phantom majorant.
constexpr int kMaxCells = 4096;
struct CellView {
    const uint32_t* q;
    int nx, ny, nz, shift;
};

template <typename R>
struct KernelArgs {
    PhantomView<R> ph;
    CellView cell;
    TableView<R> tab;
    ParamView<R> prm;
    QueueView<R> qin;     // consumed by a transport kernel
    QueueView<R> qe_out;  // electrons and positrons are appended here
    QueueView<R> qp_out;  // photons are appended here
    TallyView tally;
    StatsView stats;
    SourceView<R> src;
    TraceView trace;
    const RunDesc* run;
    uint64_t src_begin;   // first job history of this source chunk
    uint32_t src_count;
    // source order (Sec. 2.2.1, Table 1: source particles are simulated energy
    // bin by energy bin): [kSrcGroups] particles per energy group, then
    // [kSrcGroups] each group's next slot; NULL: history order
    uint32_t* src_order;
    int chunk;            // records a wave takes from the input queue at once
    int min_grid;         // fewest work-groups a transport generation keeps
    int spill_lanes;      // a wave with at most this many live lanes left sets them aside (0: off)
    int event_lanes;      // waiting electrons that start a deferred-event pass
};

// LDS bytes a transport work-group stages: the tables of every material the
// phantom holds, or (gtab: the per-material tables read from global memory,
// through L2) only the photon majorant, the scattering table and R(E_abs).
// (cells: the cell scales staged too, one byte each, for photon_mode 1)
template <typename R>
inline size_t photon_lds_bytes(int n_mats, bool gtab = false, int cells = 0)
{
    return (gtab ? 0 : 4 * sizeof(R) * size_t(n_mats) * kTabNE) + sizeof(R) * kTabNE +
           ((size_t(cells) + 15) & ~size_t(15));
}
template <typename R>
inline size_t electron_lds_bytes(int n_mats, bool gtab = false)
{
    return (gtab ? 0
                 : 2 * sizeof(R) * size_t(n_mats) * kTabNE + sizeof(R) * size_t(n_mats) * kTabNE +
                       sizeof(uint16_t) * size_t(n_mats) * kRangeCells) +
           sizeof(R) * kTabNA + sizeof(R) * ((size_t(n_mats) + 7) & ~size_t(7));
}

// Test-only sampler (omc_debug_sample): one interaction per work-item.
enum SampleKind : int {
    SMP_COMPTON = 0,
    SMP_MOLLER,
    SMP_BREMS,
    SMP_MS,
    SMP_ANNIHILATION,
    SMP_PAIR,
    SMP_SOURCE
};
constexpr int kSampleWords = 16;
struct SampleArgs {
    int which;
    uint32_t seed, n;
    double E, u, v, w;  // the particle before the event
    double x;           // multiple scattering: s / lambda_1 of the step
};

// Energy groups of the ordered source: quarter octaves of the FP32 energy
// (its bit pattern shifted right by 21: exponent and two mantissa bits, a
// monotone integer function), group 0 the highest; 0.01-20 MeV spans 44.
constexpr int kSrcGroups = 64;
constexpr int kSrcOrderItems = 16;  // histories per work-item of the ordered source passes
constexpr uint32_t kSrcGroupLo = 0x3C23D70Au >> 21;  // FP32 bits of 0.01 MeV

// Host-side launchers (one instantiation per precision).
template <typename R>
struct Launch {
    static int prepare(size_t lds_ph, size_t lds_el, bool gtab);
    // one work-item per history, or (a.src_order) per kSrcOrderItems histories
    static int source(const KernelArgs<R>& a, int grid, int block, void* stream);
    // particles per energy group of the chunk (ordered source): into a.src_order;
    // kSrcOrderItems histories per work-item
    static int source_groups(const KernelArgs<R>& a, int grid, void* stream);
    // cells: flights with a majorant per macro cell (photon_mode 1)
    static int photon(const KernelArgs<R>& a, int grid, int block, size_t lds, bool gtab,
                      bool cells, void* stream);
    // fixed: steps across voxels (electron_mode 1), a kernel of its own
    static int electron(const KernelArgs<R>& a, int grid, int block, size_t lds, bool fixed,
                        bool gtab, void* stream);
    static int sample(const KernelArgs<R>& a, const SampleArgs& sa, double* out,
                      uint32_t* words, void* stream);
};

// grid [B][copies][nvox]: the copies of a batch are summed (in order) first
int launch_fold(const double* grid, const float* rho, size_t nvox, int B, int copies,
                const double* nb, double V, double n_total, double* dose, double* dose2,
                void* stream);
int launch_queue_reset(uint32_t* ctrl, int which_mask, void* stream);
// ordered source: cursor[g] = sum of counts[g'] for g' < g, then counts zeroed
int launch_source_scan(uint32_t* order, void* stream);
// count of queue `which` += add (appends a source chunk written past the
// records already waiting in that queue)
int launch_queue_commit(uint32_t* ctrl, int which, uint32_t add, void* stream);
// zero n 64-bit words (a kernel, so that it can sit inside a captured graph)
int launch_zero(void* p, size_t n_words, void* stream);
// Sum the per-work-group statistics rows into row 0.
int launch_stats_reduce(unsigned long long* counters, double* energies, uint32_t n_rows,
                        void* stream);
constexpr uint32_t kStatsRows = 1024;

// Batched-beamlet output: the dense FP64 grid of each beam in a group is
// compacted to CSR rows of (voxel u32, dose f32) in three passes over tiles of
// kCompactTile voxels: per-tile counts, an exclusive scan of the counts (the
// output offsets, in beam-major then voxel order), and the ordered write.
// scale[b] = 1 / (V * n_b) turns a cell energy into MeV/g per history of beam
// b once divided by the voxel density; a voxel is kept when its dose is
// non-zero and above thr[b].
constexpr int kCompactTile = 2048;
int launch_beam_max(const double* grid, const float* rho, size_t nvox, int n_beams,
                    const double* scale, float* dmax, void* stream);
int launch_compact_count(const double* grid, const float* rho, size_t nvox, int n_beams,
                         const double* scale, const float* thr, uint32_t* tile_cnt, void* stream);
// exclusive scan of n counts into out[0..n] (out[n] = total); tmp holds
// (n + 1023) / 1024 + 1 words
int launch_scan(const uint32_t* in, uint64_t* out, size_t n, uint64_t* tmp, void* stream);
int launch_compact_write(const double* grid, const float* rho, size_t nvox, int n_beams,
                         const double* scale, const float* thr, const uint64_t* tile_off,
                         uint64_t nnz, uint32_t* voxel, float* dose, void* stream);
// Phase-space records checked on the device as the host checks its copies:
// out[0] += 1 and out[1] = min(out[1], k) for every bad record k (energy not in
// (0, ehi), a non-finite position or direction component, a zero direction).
int launch_check_records(const float* rec, uint32_t n, double ehi, uint32_t* out, void* stream);
// Phantom (phantom_kernels.hip): vox[v] = {rho[v] bits, slot[mat[v]]}; and the
// CT mapping of nvox HU values into rho and mat (library ids) with the largest
// density bits of each material atomically raised in rmax_bits[kMaxMaterials].
// map holds n_nodes HU nodes, n_nodes densities, n_bins bin upper bounds and
// n_nodes - 1 segment slopes.
int launch_build_vox(const float* rho, const uint8_t* mat, size_t nvox, const uint32_t* slot,
                     uint32_t* vox, void* stream);
// Cell scales: q[cell] = max over its voxels of min(255, max(1, ceil(255 *
// (rho * r[slot])))), r[slot] the largest ratio of the material's attenuation
// to the phantom majorant over the energy nodes (q zeroed before).
int launch_cell_scales(const uint32_t* vox, int nx, int ny, int nz, int shift, int cnx, int cny,
                       const double* r, uint32_t* q, void* stream);
// The mapping goes through a table of every int16 HU value (lut_rho f32 and
// lut_mat u8, kCtLutSize entries each, indexed by HU + kCtLutSize / 2).
constexpr int kCtLutSize = 65536;
int launch_ct_map(const int16_t* hu, size_t nvox, const double* map, const uint32_t* bin_mat,
                  int n_nodes, int n_bins, float* lut_rho, uint8_t* lut_mat, float* rho,
                  uint8_t* mat, uint32_t* rmax_bits, void* stream);
int launch_philox_debug(uint32_t seed, uint32_t h, uint64_t q, uint32_t n0, uint32_t nblocks,
                        uint32_t* out, void* stream);

}  // namespace omc
