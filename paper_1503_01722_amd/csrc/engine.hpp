// engine.hpp -- data shared by the host runtime and the gfx950 kernels.
//
// Layout in HBM (all allocations made once per context, sized for the run):
//   phantom     rho f32[nvox], mat u8[nvox]                x fastest
//   tables      photon  R4[n_mats][NE]  {mu_tot, mu_C, mu_PE, 0}   (cm^2/g)
//               majorant R[NE]                                     (1/cm)
//               electron R4[n_mats][NE] {R, sigma_hat, sigma_M, sigma_B}
//               K1 R[n_mats][NE], ms log2 A R[NA], R(E_abs) R[n_mats]
//   queues      four structure-of-arrays particle queues (photon cur/next,
//               electron cur/next), each {x,y,z,u,v,w,E} R, voxel u32 packed
//               (ix | iy<<10 | iz<<20), history u32, particle id 2 x u32,
//               type u8; a control block of {count, head} per queue
//   tally       B batch grids f64[B][nvox] (the one FP64 step on the GPU)
//   counters    u64[kNumCounters] and f64 energies[kNumEnergies]
// R is float for production transport and double for the parity build.
#pragma once

#include <cstddef>
#include <cstdint>

namespace omc {

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
    kNumCounters
};

enum Energy : int { EN_INCIDENT = 0, EN_DEPOSITED, EN_ESCAPED, kNumEnergies };

enum PType : int { PT_PHOTON = 0, PT_ELECTRON = 1, PT_POSITRON = 2 };

constexpr uint32_t kResBlockSlots = 128;  // output slots a wave reserves per atomic
constexpr int kTabNE = 512;
constexpr int kTabNA = 512;

template <typename R>
struct QueueView {
    R *x, *y, *z, *u, *v, *w, *E;
    uint32_t* vox;
    uint32_t* hist;
    uint32_t* qlo;
    uint32_t* qhi;
    uint8_t* type;
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
};

template <typename R>
struct TableView {
    const R* ph;      // [n_mats][NE][4]
    const R* muhat;   // [NE]
    const R* el;      // [n_mats][NE][4]
    const R* K1;      // [n_mats][NE]
    const R* msA;     // [NA]
    const R* Rabs;    // [n_mats]
    int n_mats;
    R L0, DL, INV;    // energy grid
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
    double* grid;        // [B][nvox]
    size_t nvox;
    uint64_t n_total;    // histories of the run
    uint32_t h0;
    int B;
};

struct StatsView {
    unsigned long long* counters;  // [n_rows][kNumCounters], summed at the end of a run
    double* energies;              // [n_rows][kNumEnergies]
    uint32_t n_rows;
    uint32_t* overflow;            // set to 1 when a push found its queue full
    uint32_t* max_steps;           // longest particle (steps) of the run
};

template <typename R>
struct SourceView {
    const double* cdf;   // n_bins, FP64 running sum normalised by its last entry
    const R* edges;      // n_bins + 1
    int n_bins;
    int particle;        // 0 photon, 1 electron
    int point;           // 1 point source
    R mono_E;
    R ssd, z_field, fx, fy, cx, cy, sx, sy;
    int rotate;          // gantry != 0
    R cg, sg, iso_x, iso_z;  // cos/sin of the gantry angle (host FP64)
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

template <typename R>
struct KernelArgs {
    PhantomView<R> ph;
    TableView<R> tab;
    ParamView<R> prm;
    QueueView<R> qin;     // consumed by a transport kernel
    QueueView<R> qe_out;  // electrons and positrons are appended here
    QueueView<R> qp_out;  // photons are appended here
    TallyView tally;
    StatsView stats;
    SourceView<R> src;
    TraceView trace;
    uint32_t seed;
    uint32_t src_begin;   // first history of this source chunk (relative to h0)
    uint32_t src_count;
    int chunk;            // records a wave takes from the input queue at once
};

// LDS bytes a transport work-group stages (tables of all materials).
template <typename R>
inline size_t photon_lds_bytes(int n_mats)
{
    return 4 * sizeof(R) * size_t(n_mats) * kTabNE + sizeof(R) * kTabNE;
}
template <typename R>
inline size_t electron_lds_bytes(int n_mats)
{
    return 4 * sizeof(R) * size_t(n_mats) * kTabNE + sizeof(R) * size_t(n_mats) * kTabNE +
           sizeof(R) * kTabNA + sizeof(R) * 8;
}

// Host-side launchers (one instantiation per precision).
template <typename R>
struct Launch {
    static int source(const KernelArgs<R>& a, int grid, int block, void* stream);
    static int photon(const KernelArgs<R>& a, int grid, int block, size_t lds, void* stream);
    static int electron(const KernelArgs<R>& a, int grid, int block, size_t lds, void* stream);
};

int launch_fold(const double* grid, const float* rho, size_t nvox, int B, const double* nb,
                double V, double n_total, double* dose, double* dose2, void* stream);
int launch_queue_reset(uint32_t* ctrl, int which_mask, void* stream);
// Sum the per-work-group statistics rows into row 0.
int launch_stats_reduce(unsigned long long* counters, double* energies, uint32_t n_rows,
                        void* stream);
constexpr uint32_t kStatsRows = 1024;
int launch_philox_debug(uint32_t seed, uint32_t h, uint64_t q, uint32_t n0, uint32_t nblocks,
                        uint32_t* out, void* stream);

}  // namespace omc
