// runtime.cpp -- host runtime and C ABI (include/omc.h) of the gfx950 engine.
//
// One context per phantom. A run transports a job: a list of beams (one for
// omc_run, one per beamlet for omc_run_beamlets) whose histories are numbered
// 0 .. N-1 across the beams and tallied in cells (batches, or beamlets):
//   for each chunk of job histories:
//     source kernel -> photon or electron queue (after what is waiting there)
//     generations: photon kernel (photon queue -> electrons, annihilation
//                  photons, the photon itself until it is absorbed or leaves)
//                  electron kernel (electron queue -> deltas, bremsstrahlung
//                  and annihilation photons); swap queues
//   then fold the batch cells into dose and dose^2, or compact the beamlet
//   cells into sparse rows.
// The paper picks the largest of {photon stack, electron stack, source} per
// iteration and launches M same-type work-items; here each generation drains a
// whole queue with a persistent grid that keeps every lane busy. Generations
// are either driven from the host (queue counts read back after each, until
// both queues are empty) or captured once as a HIP graph with a fixed number
// of generations per chunk: the kernels size themselves from the counts on the
// device, particles left after a chunk's generations join the next chunk's,
// and the host drains what the last chunk leaves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/omc.h"
#include "engine.hpp"
#include "tables.hpp"

namespace {

thread_local std::string g_thread_error;

template <typename R>
struct DeviceTables {
    R* ph = nullptr;
    R* muhat = nullptr;
    R* el = nullptr;
    R* hard = nullptr;
    R* rtab = nullptr;
    uint16_t* ridx = nullptr;
    R* msA = nullptr;
    R* Rabs = nullptr;
    R* edges = nullptr;
    uint32_t rshift = 0, rbase = 0, rcells = 1;
    // macro-cell majorant scales (photon_mode 1), built with the tables
    uint32_t* cellq = nullptr;
    double* cell_r = nullptr;
    int cnx = 1, cny = 1, cnz = 1, cshift = 0;
    bool cells_valid = false;  // built on the first photon_mode 1 run after the tables
    bool valid = false;
};

template <typename R>
struct DeviceQueues {
    void* mem = nullptr;
    size_t bytes = 0;
    uint32_t cap_ph = 0, cap_el = 0;
    omc::QueueView<R> q[4] = {};  // 0,1 photon buffers; 2,3 electron buffers
};

}  // namespace

struct omc_ctx {
    int device = 0;
    int nx = 0, ny = 0, nz = 0;
    double dx = 0, dy = 0, dz = 0;
    size_t nvox = 0;
    std::vector<omc::MaterialSpec> mats;
    std::vector<double> rho_max;  // per material
    // table slots: the device tables hold the materials present in the phantom
    // only, in library order; the voxel records carry the slot
    std::vector<int> present;     // slot -> library material
    std::vector<uint32_t> slot_of;  // library material -> slot (absent: 0)
    bool last_gtab = false;       // the last run read its tables from global memory

    bool has_source = false;
    std::vector<float> psf;  // phase-space records of the source (geometry 2)
    omc_source src{};
    std::vector<double> edges, weights, cdf;
    omc_params prm{};

    int cu_count = 0;
    float* d_rho = nullptr;
    uint8_t* d_mat = nullptr;
    uint32_t* d_vox = nullptr;  // [nvox][2]: density bits, table slot
    uint32_t* d_slot = nullptr;  // [kMaxMaterials] slot of each library material
    double* d_grid = nullptr;
    size_t grid_cells = 0;      // tally cells d_grid holds (nvox doubles each)
    char* d_src = nullptr;      // beams, history prefix, spectra of the current job
    size_t src_cap = 0;
    std::vector<char> src_stage;  // host copy of d_src, alive until the run's end
    float* d_psf = nullptr;     // device copy of psf, uploaded once per omc_set_source
    const float* psf_dev = nullptr;  // the caller's device records (psf_on_device), not owned
    uint32_t* d_chk = nullptr;  // [2] result of the device record check
    size_t psf_cap = 0;         // floats d_psf holds
    bool psf_dirty = true;
    omc::RunDesc* d_run = nullptr;
    uint32_t* d_order = nullptr;  // [2 kSrcGroups]: ordered source counts and cursors
    omc::RunDesc* h_run = nullptr;  // pinned
    double* d_dose = nullptr;   // fold target of omc_run
    double* d_dose2 = nullptr;
    uint32_t* d_ctrl = nullptr;  // [4][count, head], overflow at [8]
    unsigned long long* d_counters = nullptr;
    double* d_energies = nullptr;
    uint32_t* h_ctrl = nullptr;  // pinned readback
    char* d_scratch = nullptr;   // this device's copy of the fixed scratch array (or NULL)

    // host-side tables (FP64) for the current Wcc, kc, Eabs_e
    std::vector<omc::MaterialTables> tabs;
    std::array<double, omc::kNA> ms{};
    double tab_Wcc = -1, tab_kc = -1, tab_Eabs = -1;
    std::vector<double> Rabs;

    DeviceTables<float> t32;
    DeviceTables<double> t64;
    DeviceQueues<float> q32;
    DeviceQueues<double> q64;

    // captured launch sequence of the last graph-mode job
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    std::vector<unsigned char> graph_key;
    int graph_pc = 0, graph_ec = 2;  // current queues after the graph
    uint32_t graph_iters = 0;

    // beamlet compaction scratch
    char* d_cscratch = nullptr;
    size_t cscratch_cap = 0;

    omc_counters last{};
    omc_timing timing{};
    omc::TraceView trace{};
    std::string err;
};

namespace {

int fail(omc_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    g_thread_error = msg;
    return code;
}

int hip_fail(omc_ctx* c, hipError_t e, const char* what)
{
    return fail(c, OMC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

template <typename T>
void dfree(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <typename R>
void free_tables(DeviceTables<R>& t)
{
    dfree(t.ph);
    dfree(t.muhat);
    dfree(t.el);
    dfree(t.hard);
    dfree(t.rtab);
    dfree(t.ridx);
    dfree(t.msA);
    dfree(t.Rabs);
    dfree(t.edges);
    t.valid = false;
    dfree(t.cellq);
    dfree(t.cell_r);
}

template <typename R>
void free_queues(DeviceQueues<R>& q)
{
    if (q.mem) (void)hipFree(q.mem);
    q = DeviceQueues<R>{};
}

int validate_material(const omc_material& m, omc::MaterialSpec& out, std::string& why)
{
    if (m.n_elem < 1 || m.n_elem > 32 || !m.Z || !m.A || !m.w_mass) {
        why = "material needs 1..32 elements with Z, A and w_mass";
        return OMC_EINVAL;
    }
    if (!finite_pos(m.I_eV) || !finite_pos(m.rho_nominal)) {
        why = "material I_eV and rho_nominal must be finite and > 0";
        return OMC_EINVAL;
    }
    out.elements.clear();
    double wsum = 0;
    for (int j = 0; j < m.n_elem; ++j) {
        if (m.Z[j] < 1 || m.Z[j] > 100 || !finite_pos(m.A[j]) || !(m.w_mass[j] >= 0) ||
            !std::isfinite(m.w_mass[j])) {
            why = "element with invalid Z, A or mass fraction";
            return OMC_EINVAL;
        }
        out.elements.push_back({m.Z[j], m.A[j], m.w_mass[j]});
        wsum += m.w_mass[j];
    }
    if (!(wsum > 0)) {
        why = "mass fractions sum to zero";
        return OMC_EINVAL;
    }
    out.I_eV = m.I_eV;
    out.rho_nominal = m.rho_nominal;
    return OMC_OK;
}

void host_tables(omc_ctx* c)
{
    if (c->tab_Wcc == c->prm.Wcc && c->tab_kc == c->prm.kc && c->tab_Eabs == c->prm.Eabs_e) return;
    c->tabs.clear();
    c->Rabs.clear();
    for (const auto& m : c->mats) {
        c->tabs.push_back(omc::build_material_tables(m, c->prm.Wcc, c->prm.kc));
        c->Rabs.push_back(omc::lerp_log2(c->tabs.back().R, c->prm.Eabs_e));
    }
    c->ms = omc::build_ms_table();
    c->tab_Wcc = c->prm.Wcc;
    c->tab_kc = c->prm.kc;
    c->tab_Eabs = c->prm.Eabs_e;
    c->t32.valid = false;
    c->t64.valid = false;
}

template <typename R>
int upload(omc_ctx* c, R*& dst, const std::vector<R>& v)
{
    dfree(dst);
    if (v.empty()) return OMC_OK;
    if (hipMalloc(&dst, v.size() * sizeof(R)) != hipSuccess)
        return fail(c, OMC_ENOMEM, "hipMalloc failed for a table");
    HIP_TRY(c, hipMemcpy(dst, v.data(), v.size() * sizeof(R), hipMemcpyHostToDevice));
    return OMC_OK;
}

// Index of the range inverse: cell k of the range axis holds the FP32 values
// whose bit pattern, shifted right by rshift, equals rbase + k (positive floats
// order as their bit patterns, so cells are monotone in R and each spans
// 1/2^(23-rshift) of an octave). The entry is the largest node j <= NE-2 with
// R_j at or below the cell's smallest value; the device walks from there to
// the exact bracket. The axis starts at R_1 (the range vanishes at the lowest
// energy node, and every value below R_1 falls in the first cell); the shift
// is the smallest that fits every material's axis in kRangeCells cells.
template <typename R>
void range_index(const std::vector<R>& rtab, int nm, DeviceTables<R>& t,
                 std::vector<uint16_t>& ridx)
{
    const int NE = omc::kNE;
    auto bits = [](double v) {
        const float f = float(v);
        uint32_t b;
        std::memcpy(&b, &f, sizeof b);
        return b;
    };
    uint32_t lo = ~0u, hi = 0u;
    for (int m = 0; m < nm; ++m) {
        lo = std::min(lo, bits(double(rtab[size_t(m) * NE + 1])));  // R_0 = 0
        hi = std::max(hi, bits(double(rtab[size_t(m) * NE + NE - 1])));
    }
    uint32_t shift = 8;
    while (((hi >> shift) - (lo >> shift)) + 1 > uint32_t(omc::kRangeCells)) ++shift;
    t.rshift = shift;
    t.rbase = lo >> shift;
    t.rcells = (hi >> shift) - t.rbase + 1;
    ridx.assign(size_t(nm) * omc::kRangeCells, 0);
    for (int m = 0; m < nm; ++m) {
        const R* r = rtab.data() + size_t(m) * NE;
        int j = 0;
        for (uint32_t k = 0; k < uint32_t(omc::kRangeCells); ++k) {
            const uint32_t cb = (t.rbase + std::min(k, t.rcells - 1)) << shift;
            float cf;
            std::memcpy(&cf, &cb, sizeof cf);
            while (j < NE - 2 && double(r[j + 1]) <= double(cf)) ++j;
            ridx[size_t(m) * omc::kRangeCells + k] = uint16_t(j);
        }
    }
}

// Ratio of each present material's attenuation per unit density to the
// photon majorant, largest over the energy nodes (indexed by table slot): a
// voxel of density rho and slot k attenuates at most rho r[k] times the
// majorant at any energy (both are interpolated linearly between the same
// nodes).
std::vector<double> majorant_ratios(const omc_ctx* c)
{
    const int NE = omc::kNE;
    std::vector<double> mh(NE, 0.0);
    for (int i = 0; i < NE; ++i)
        for (int m : c->present) mh[i] = std::max(mh[i], c->rho_max[m] * c->tabs[m].muTot[i]);
    std::vector<double> r(omc::kMaxMaterials, 0.0);
    for (size_t k = 0; k < c->present.size(); ++k)
        for (int i = 0; i < NE; ++i) {
            const double q = c->tabs[c->present[k]].muTot[i] / mh[i];
            if (mh[i] > 0.0 && q > r[k]) r[k] = q;
        }
    return r;
}

// Macro cells for the photon majorant per cell (photon_mode 1): the smallest
// power-of-two side that leaves at most kMaxCells cells; each cell's scale is
// the largest over its voxels of rho * r_m in 255ths, rounded up, r_m the
// largest ratio of material m's attenuation to the majorant over the nodes.
template <typename R>
int cell_scales(omc_ctx* c, DeviceTables<R>& t)
{
    t.cshift = 0;
    for (;;) {
        t.cnx = (c->nx + (1 << t.cshift) - 1) >> t.cshift;
        t.cny = (c->ny + (1 << t.cshift) - 1) >> t.cshift;
        t.cnz = (c->nz + (1 << t.cshift) - 1) >> t.cshift;
        if (size_t(t.cnx) * t.cny * t.cnz <= size_t(omc::kMaxCells)) break;
        t.cshift += 1;
    }
    const std::vector<double> r = majorant_ratios(c);
    if (!t.cellq && hipMalloc(&t.cellq, omc::kMaxCells * sizeof(uint32_t)) != hipSuccess) {
        t.cellq = nullptr;
        return fail(c, OMC_ENOMEM, "hipMalloc failed for the cell scales");
    }
    if (!t.cell_r && hipMalloc(&t.cell_r, omc::kMaxMaterials * sizeof(double)) != hipSuccess) {
        t.cell_r = nullptr;
        return fail(c, OMC_ENOMEM, "hipMalloc failed for the cell scales");
    }
    const std::vector<uint32_t> zero(omc::kMaxCells, 0u);
    HIP_TRY(c, hipMemcpy(t.cellq, zero.data(), zero.size() * sizeof(uint32_t),
                         hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(t.cell_r, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice));
    if (omc::launch_cell_scales(c->d_vox, c->nx, c->ny, c->nz, t.cshift, t.cnx, t.cny, t.cell_r,
                                t.cellq, nullptr))
        return fail(c, OMC_EDEVICE, "cell scale launch failed");
    HIP_TRY(c, hipStreamSynchronize(nullptr));
    return OMC_OK;
}

template <typename R>
int device_tables(omc_ctx* c, DeviceTables<R>& t)
{
    host_tables(c);
    if (t.valid) return OMC_OK;
    const int nm = int(c->present.size());
    const int NE = omc::kNE;
    std::vector<R> ph(size_t(nm) * NE * 4), el(size_t(nm) * NE * 2), hard(size_t(nm) * NE * 2),
        rtab(size_t(nm) * NE), muhat(NE), msA(omc::kNA), Rabs(nm);
    for (int m = 0; m < nm; ++m) {
        const auto& T = c->tabs[c->present[m]];
        for (int i = 0; i < NE; ++i) {
            const size_t o = (size_t(m) * NE + i) * 4;
            ph[o + 0] = R(T.muTot[i]);
            ph[o + 1] = R(T.muC[i]);
            ph[o + 2] = R(T.muPE[i]);
            ph[o + 3] = R(0);
            const size_t o2 = (size_t(m) * NE + i) * 2;
            el[o2 + 0] = R(T.K1[i]);
            el[o2 + 1] = R(T.sigHat[i]);
            hard[o2 + 0] = R(T.sigM[i]);
            hard[o2 + 1] = R(T.sigB[i]);
            rtab[size_t(m) * NE + i] = R(T.R[i]);
        }
        Rabs[m] = R(c->Rabs[c->present[m]]);
    }
    // photon majorant over the materials present: node-wise max of
    // rho_max(m) * mu_tot(m), whose interpolant bounds every material's
    for (int i = 0; i < NE; ++i) {
        double mx = 0.0;
        for (int m : c->present) mx = std::max(mx, c->rho_max[m] * c->tabs[m].muTot[i]);
        muhat[i] = R(mx);
    }
    for (int j = 0; j < omc::kNA; ++j) msA[j] = R(c->ms[j]);
    std::vector<uint16_t> ridx;
    range_index(rtab, nm, t, ridx);
    int rc;
    if ((rc = upload(c, t.ph, ph)) || (rc = upload(c, t.el, el)) || (rc = upload(c, t.hard, hard)) ||
        (rc = upload(c, t.rtab, rtab)) || (rc = upload(c, t.ridx, ridx)) ||
        (rc = upload(c, t.muhat, muhat)) || (rc = upload(c, t.msA, msA)) ||
        (rc = upload(c, t.Rabs, Rabs)))
        return rc;
    t.cells_valid = false;
    t.valid = true;
    return OMC_OK;
}

// Records a queue may hold: each of its arrays stays below 4 GiB, so that the
// kernels address a record's fields by 32-bit byte offsets (a multiple of 64)
template <typename R>
constexpr uint64_t queue_records_max()
{
    return ((uint64_t(1) << 32) / sizeof(R) - 64) & ~uint64_t(63);
}

template <typename R>
int ensure_queues(omc_ctx* c, DeviceQueues<R>& Q, uint32_t cap_ph, uint32_t cap_el)
{
    if (Q.mem && Q.cap_ph >= cap_ph && Q.cap_el >= cap_el) return OMC_OK;
    free_queues(Q);
    // capacities in multiples of 64 records keep every array 256-byte aligned
    // with no padding between arrays, so the layout below is exactly `bytes`
    cap_ph = uint32_t(std::min<uint64_t>((uint64_t(cap_ph) + 63) & ~uint64_t(63), queue_records_max<R>()));
    cap_el = uint32_t(std::min<uint64_t>((uint64_t(cap_el) + 63) & ~uint64_t(63), queue_records_max<R>()));
    const size_t per = 8 * sizeof(R) + 6 * sizeof(uint32_t);
    const size_t bytes = (size_t(cap_ph) * 2 + size_t(cap_el) * 2) * per;
    if (hipMalloc(&Q.mem, bytes) != hipSuccess) {
        Q.mem = nullptr;
        return fail(c, OMC_ENOMEM, "hipMalloc failed for the particle queues");
    }
    Q.bytes = bytes;
    Q.cap_ph = cap_ph;
    Q.cap_el = cap_el;
    char* p = static_cast<char*>(Q.mem);
    auto take = [&p](size_t n) {
        char* r = p;
        p += (n + 255) & ~size_t(255);
        return r;
    };
    for (int k = 0; k < 4; ++k) {
        const uint32_t cap = k < 2 ? cap_ph : cap_el;
        omc::QueueView<R>& q = Q.q[k];
        q.x = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q.y = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q.z = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q.u = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q.v = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q.w = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q.E = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q.vox = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q.hist = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q.qlo = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q.qhi = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q.tag = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q.aux_pos = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q.aux_f = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q.cap = cap;
        q.count = c->d_ctrl + 2 * k;
        q.head = c->d_ctrl + 2 * k + 1;
    }
    if (size_t(p - static_cast<char*>(Q.mem)) != bytes) {
        free_queues(Q);
        return fail(c, OMC_EUNSUP, "internal error: queue layout does not match its allocation");
    }
    return OMC_OK;
}

void batch_sizes(uint64_t N, int B, std::vector<double>& nb)
{
    nb.assign(B, 0.0);
    for (int b = 0; b < B; ++b) {
        const uint64_t i0 = (uint64_t(b) * N + uint64_t(B) - 1) / uint64_t(B);
        const uint64_t i1 = (uint64_t(b + 1) * N + uint64_t(B) - 1) / uint64_t(B);
        nb[b] = double(i1 - i0);
    }
}

// HIP events around eager launches (read and destroyed at the end of a run).
struct EventTimer {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
    void begin(int kind)
    {
        if (!on) return;
        hipEvent_t a = nullptr, b = nullptr;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, s);
        ev.push_back({kind, {a, b}});
    }
    void end()
    {
        if (!on) return;
        (void)hipEventRecord(ev.back().second.second, s);
    }
};

void collect_events(std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>& ev,
                    omc_timing& t)
{
    for (auto& e : ev) {
        float ms = 0;
        (void)hipEventSynchronize(e.second.second);
        (void)hipEventElapsedTime(&ms, e.second.first, e.second.second);
        t.launches[e.first] += 1;
        t.total_ms[e.first] += ms;
    }
    (void)hipGetLastError();  // a failed event query must not look like a failed launch later
}

void destroy_events(std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>& ev)
{
    for (auto& e : ev) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    ev.clear();
}

// whole-run wall time on the device: events recorded before the first and
// after the last launch of a run
struct RunClock {
    hipEvent_t a = nullptr, b = nullptr;
    void start(bool on, hipStream_t s)
    {
        if (!on) return;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, s);
    }
    void stop(hipStream_t s)
    {
        if (a) (void)hipEventRecord(b, s);
    }
    void collect(omc_timing& t)
    {
        if (!a) return;
        float ms = 0;
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&ms, a, b);
        t.run_ms = ms;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        a = b = nullptr;
    }
};

void drop_graph(omc_ctx* c)
{
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    c->graph_key.clear();
}

int check_ctx(const omc_ctx* c) { return c ? OMC_OK : OMC_EINVAL; }

DeviceTables<float>& tables_of(omc_ctx* c, float) { return c->t32; }
DeviceTables<double>& tables_of(omc_ctx* c, double) { return c->t64; }
DeviceQueues<float>& queues_of(omc_ctx* c, float) { return c->q32; }
DeviceQueues<double>& queues_of(omc_ctx* c, double) { return c->q64; }

// counters in the order of omc::Counter
uint64_t omc_counters::*const kCounterField[omc::kNumCounters] = {
    &omc_counters::ph_flights,  &omc_counters::ph_fictitious, &omc_counters::ph_compton,
    &omc_counters::ph_photo,    &omc_counters::ph_pair,       &omc_counters::ph_cutoff,
    &omc_counters::ph_escaped,  &omc_counters::el_steps,      &omc_counters::el_hard_cand,
    &omc_counters::el_hard_fict, &omc_counters::el_moller,    &omc_counters::el_brems,
    &omc_counters::el_absorbed, &omc_counters::el_escaped,    &omc_counters::el_boundary,
    &omc_counters::el_hinge_trunc, &omc_counters::pos_annihil, &omc_counters::push_ph,
    &omc_counters::push_el,     &omc_counters::src_miss,      &omc_counters::watchdog,
    &omc_counters::set_aside};

// ------------------------------------------------------------------- sources
// Checks a source as omc_set_source documents and returns its spectrum as bin
// edges and the normalised FP64 running sum of the weights.
// Host records are checked and copied into *psf (skipped when psf is null: the
// caller has them already); device records are checked by check_device_records.
int check_source(const omc_source* s, std::vector<double>& edges, std::vector<double>& cdf,
                 std::vector<float>* psf, std::string& why)
{
    edges.clear();
    cdf.clear();
    if (psf) psf->clear();
    if (!s) {
        why = "NULL source";
        return OMC_EINVAL;
    }
    if (s->particle != 0 && s->particle != 1) {
        why = "particle must be 0 or 1";
        return OMC_EINVAL;
    }
    if (s->geometry < 0 || s->geometry > 2) {
        why = "geometry must be 0, 1 or 2";
        return OMC_EINVAL;
    }
    if (s->geometry == 2) {
        // phase space: records checked and copied; spectrum and field unused
        if (s->n_psf < 1 || s->n_psf > (1 << 26) || !s->psf) {
            why = "a phase space needs 1 <= n_psf <= 2^26 records";
            return OMC_EINVAL;
        }
        const double chk[] = {s->gantry_deg, s->iso_x, s->iso_z};
        for (double v : chk)
            if (!std::isfinite(v)) {
                why = "non-finite source geometry";
                return OMC_EINVAL;
            }
        if (s->psf_on_device != 0 && s->psf_on_device != 1) {
            why = "psf_on_device must be 0 or 1";
            return OMC_EINVAL;
        }
        if (s->psf_on_device || !psf) return OMC_OK;
        psf->assign(s->psf, s->psf + size_t(s->n_psf) * 8);
        for (int k = 0; k < s->n_psf; ++k) {
            const float* r = psf->data() + size_t(k) * 8;
            bool ok = r[0] > 0.0f && double(r[0]) < omc::kEHi;
            for (int j = 1; j < 7; ++j) ok = ok && std::isfinite(r[j]);
            const double n2 = double(r[4]) * r[4] + double(r[5]) * r[5] + double(r[6]) * r[6];
            if (!ok || !(n2 > 1e-12)) {
                why = "phase-space record " + std::to_string(k) +
                      ": energy must be in (0, 20) MeV, position finite, direction non-zero";
                return OMC_EINVAL;
            }
        }
        return OMC_OK;
    }
    if (!(s->fx > 0) || !(s->fy > 0) || !std::isfinite(s->fx) || !std::isfinite(s->fy)) {
        why = "field size must be > 0";
        return OMC_EINVAL;
    }
    if (s->geometry == 1 && !finite_pos(s->ssd)) {
        why = "ssd must be > 0";
        return OMC_EINVAL;
    }
    const double chk[] = {s->z_field, s->cx, s->cy, s->sx, s->sy, s->gantry_deg, s->iso_x, s->iso_z};
    for (double v : chk)
        if (!std::isfinite(v)) {
            why = "non-finite source geometry";
            return OMC_EINVAL;
        }
    if (s->n_bins < 0 || s->n_bins > 4096) {
        why = "n_bins out of range";
        return OMC_EINVAL;
    }
    if (s->n_bins == 0) {
        if (!(s->mono_E > 0) || !(s->mono_E < omc::kEHi)) {
            why = "mono_E must be in (0, 20) MeV";
            return OMC_EINVAL;
        }
        return OMC_OK;
    }
    if (!s->edges || !s->weights) {
        why = "spectrum arrays are NULL";
        return OMC_EINVAL;
    }
    edges.assign(s->edges, s->edges + s->n_bins + 1);
    for (int b = 0; b <= s->n_bins; ++b)
        if (!(edges[b] > 0) || !(edges[b] < omc::kEHi) || (b && !(edges[b] > edges[b - 1]))) {
            why = "spectrum edges must increase within (0, 20) MeV";
            return OMC_EINVAL;
        }
    double acc = 0.0;
    for (int b = 0; b < s->n_bins; ++b) {
        const double w = s->weights[b];
        if (!(w >= 0) || !std::isfinite(w)) {
            why = "spectrum weights must be finite and >= 0";
            return OMC_EINVAL;
        }
        acc += w;
        cdf.push_back(acc);
    }
    if (!(acc > 0)) {
        why = "empty spectrum";
        return OMC_EINVAL;
    }
    for (double& v : cdf) v = v / acc;
    return OMC_OK;
}

// One beam of a job on the host. Spectra are shared between beams by pointer.
// Device records (psf_on_device): the pointer must lie in a HIP allocation on the
// context's device that holds all n records; then every record is checked on
// the device with the host's conditions, before any kernel reads them.
// True when [p, p + bytes) lies inside one HIP allocation of the context's
// device (a caller's device buffer, checked before any kernel reads it).
bool device_range_ok(const omc_ctx* c, const void* p, size_t bytes, size_t align)
{
    hipPointerAttribute_t at{};
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    const bool dev = hipPointerGetAttributes(&at, p) == hipSuccess &&
                     at.type == hipMemoryTypeDevice && at.device == c->device;
    const bool range =
        dev && hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess &&
        reinterpret_cast<uintptr_t>(p) >= reinterpret_cast<uintptr_t>(base) &&
        reinterpret_cast<uintptr_t>(p) + bytes <= reinterpret_cast<uintptr_t>(base) + size;
    (void)hipGetLastError();
    return dev && range && reinterpret_cast<uintptr_t>(p) % align == 0;
}

int check_device_records(omc_ctx* c, const float* p, int n, std::string& why)
{
    if (!device_range_ok(c, p, size_t(n) * 8 * sizeof(float), alignof(float))) {
        why = "psf_on_device: the records must be an allocation of this context's device "
              "holding n_psf x 8 floats";
        return OMC_EINVAL;
    }
    if (!c->d_chk && hipMalloc(&c->d_chk, 2 * sizeof(uint32_t)) != hipSuccess) {
        c->d_chk = nullptr;
        why = "hipMalloc failed for the record check";
        return OMC_ENOMEM;
    }
    uint32_t h[2] = {0u, 0xFFFFFFFFu};
    if (hipMemcpy(c->d_chk, h, sizeof h, hipMemcpyHostToDevice) != hipSuccess ||
        omc::launch_check_records(p, uint32_t(n), omc::kEHi, c->d_chk, nullptr) ||
        hipMemcpy(h, c->d_chk, sizeof h, hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        why = "the device record check failed";
        return OMC_EDEVICE;
    }
    if (h[0]) {
        why = "phase-space record " + std::to_string(h[1]) +
              ": energy must be in (0, 20) MeV, position finite, direction non-zero";
        return OMC_EINVAL;
    }
    return OMC_OK;
}

struct HostBeam {
    omc_source src;                     // spectrum and record pointers unused
    const std::vector<double>* edges;   // n_bins + 1
    const std::vector<double>* cdf;     // n_bins
    uint64_t n;
    uint32_t h0;
    const std::vector<float>* psf;      // n_psf x 8 host records (phase space), else empty
    const float* psf_dev = nullptr;     // or the caller's device records
};

struct Job {
    std::vector<HostBeam> beams;
    int particle = 0;
    int cell_mode = 0;  // 0: cells are batches of the history range; 1: cells are beams
    int cells = 1;
    uint64_t N = 0;
};

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Lay the job's beams out in device memory (one upload, asynchronous on s; the
// host copy stays alive in the context until the run has synchronised).
template <typename R>
int pack_sources(omc_ctx* c, const Job& job, hipStream_t s, omc::SourceView<R>& v,
                 char* fixed = nullptr, size_t fixed_cap = 0)
{
    const size_t nb = job.beams.size();
    std::vector<omc::BeamSrc<R>> bs(nb);
    std::vector<uint64_t> first(nb + 1, 0);
    std::vector<double> cdf;
    std::vector<R> edges;
    std::vector<float> recs;
    const std::vector<double>* last = nullptr;
    const std::vector<float>* last_psf = nullptr;
    int last_c = 0, last_e = 0, last_p = 0;
    // a run of the context's own source reads the records from their resident
    // copy (uploaded once per omc_set_source); batched beamlets bring theirs
    const bool resident = nb == 1 && job.beams[0].src.geometry == 2 &&
                          !job.beams[0].psf_dev && job.beams[0].psf == &c->psf;
    std::vector<long long> rec_at(nb, -1);  // first float of a beam's records in recs
    for (size_t b = 0; b < nb; ++b) {
        const HostBeam& hb = job.beams[b];
        const omc_source& sr = hb.src;
        omc::BeamSrc<R>& o = bs[b];
        std::memset(&o, 0, sizeof o);
        o.mono_E = R(sr.mono_E);
        o.ssd = R(sr.ssd);
        o.z_field = R(sr.z_field);
        o.fx = R(sr.fx);
        o.fy = R(sr.fy);
        o.cx = R(sr.cx);
        o.cy = R(sr.cy);
        o.sx = R(sr.sx);
        o.sy = R(sr.sy);
        const double gr = sr.gantry_deg * omc::kPi / 180.0;
        o.cg = R(std::cos(gr));
        o.sg = R(std::sin(gr));
        o.iso_x = R(sr.iso_x);
        o.iso_z = R(sr.iso_z);
        o.n_bins = sr.geometry == 2 ? 0 : sr.n_bins;
        o.point = sr.geometry == 1;
        if (sr.geometry == 2) {
            // beams given the same record array share one device copy
            if (hb.psf_dev) {
                o.n_psf = sr.n_psf;
                o.psf = hb.psf_dev;
            } else {
                if (!resident && hb.psf != last_psf) {
                    last_psf = hb.psf;
                    last_p = int(recs.size() / 8);
                    recs.insert(recs.end(), hb.psf->begin(), hb.psf->end());
                }
                o.n_psf = int(hb.psf->size() / 8);
                if (!resident) rec_at[b] = 8LL * last_p;
            }
        }
        o.rotate = sr.gantry_deg != 0.0;
        o.h0 = hb.h0;
        if (o.n_bins > 0) {
            if (hb.edges != last) {
                last = hb.edges;
                last_c = int(cdf.size());
                last_e = int(edges.size());
                cdf.insert(cdf.end(), hb.cdf->begin(), hb.cdf->end());
                for (double e : *hb.edges) edges.push_back(R(e));
            }
            o.cdf_off = last_c;
            o.edge_off = last_e;
        }
        first[b + 1] = first[b] + hb.n;
    }
    const size_t o_beams = 0;
    const size_t o_first = o_beams + align256(nb * sizeof(omc::BeamSrc<R>));
    const size_t o_cdf = o_first + align256((nb + 1) * sizeof(uint64_t));
    const size_t o_edges = o_cdf + align256(std::max<size_t>(cdf.size(), 1) * sizeof(double));
    const size_t o_psf = o_edges + align256(std::max<size_t>(edges.size(), 1) * sizeof(R));
    const size_t total = o_psf + align256(std::max<size_t>(recs.size(), 1) * sizeof(float));
    if (fixed) {
        // a run that may not allocate: the description goes into the fixed
        // buffer, and a resident phase space must be on the device already
        if (total > fixed_cap)
            return fail(c, OMC_EINVAL, "the source description exceeds the fixed scratch");
        if (resident && (c->psf_dirty || !c->d_psf))
            return fail(c, OMC_ESTATE, "the phase-space records are not on the device yet: "
                                       "run omc_run or omc_run_device once after "
                                       "omc_set_source");
    } else if (c->src_cap < total) {
        dfree(c->d_src);
        c->src_cap = 0;
        const size_t want = std::max<size_t>(total, 64 * 1024);
        if (hipMalloc(&c->d_src, want) != hipSuccess) {
            c->d_src = nullptr;
            return fail(c, OMC_ENOMEM, "hipMalloc failed for the source description");
        }
        c->src_cap = want;
    }
    if (!fixed && resident && (c->psf_dirty || !c->d_psf)) {
        if (c->psf_cap < c->psf.size()) {
            dfree(c->d_psf);
            c->psf_cap = 0;
            if (hipMalloc(&c->d_psf, c->psf.size() * sizeof(float)) != hipSuccess) {
                c->d_psf = nullptr;
                return fail(c, OMC_ENOMEM, "hipMalloc failed for the phase-space records");
            }
            c->psf_cap = c->psf.size();
        }
        // c->psf is stable until the next omc_set_source, after this run's end
        HIP_TRY(c, hipMemcpyAsync(c->d_psf, c->psf.data(), c->psf.size() * sizeof(float),
                                  hipMemcpyHostToDevice, s));
        c->psf_dirty = false;
    }
    char* const dst = fixed ? fixed : c->d_src;
    // record pointers: the resident copy, or this job's records in the description
    for (size_t b = 0; b < nb; ++b)
        if (bs[b].n_psf > 0 && !job.beams[b].psf_dev)
            bs[b].psf = rec_at[b] < 0 ? c->d_psf
                                      : reinterpret_cast<const float*>(dst + o_psf) + rec_at[b];
    c->src_stage.assign(total, 0);
    char* h = c->src_stage.data();
    std::memcpy(h + o_beams, bs.data(), nb * sizeof(omc::BeamSrc<R>));
    std::memcpy(h + o_first, first.data(), (nb + 1) * sizeof(uint64_t));
    if (!cdf.empty()) std::memcpy(h + o_cdf, cdf.data(), cdf.size() * sizeof(double));
    if (!edges.empty()) std::memcpy(h + o_edges, edges.data(), edges.size() * sizeof(R));
    if (!recs.empty()) std::memcpy(h + o_psf, recs.data(), recs.size() * sizeof(float));
    HIP_TRY(c, hipMemcpyAsync(dst, h, total, hipMemcpyHostToDevice, s));
    v.beams = reinterpret_cast<const omc::BeamSrc<R>*>(dst + o_beams);
    v.first = reinterpret_cast<const uint64_t*>(dst + o_first);
    v.cdf = reinterpret_cast<const double*>(dst + o_cdf);
    v.edges = reinterpret_cast<const R*>(dst + o_edges);
    v.n_beams = int(nb);
    v.particle = job.particle;
    v.cell_mode = job.cell_mode;
    return OMC_OK;
}

// ----------------------------------------------------------------- transport
// Transport every history of the job into the cell grids; the statistics stay
// on the device (finish_stats reads them). L.iterations counts generations.
// Device memory of a run besides the phantom and the tables: the context's
// own buffers (queues and tally grids allocated on demand), or regions of the
// library's fixed scratch array for a run that may not allocate.
struct RunMem {
    uint32_t* ctrl;                 // [64]: queue {count, head} x 4, overflow, ...
    unsigned long long* counters;   // [rows][kNumCounters]
    double* energies;               // [rows][kNumEnergies]
    uint32_t rows;
    omc::RunDesc* run;
    double* grid;                   // tally cells (set by transport for the context's own)
    uint32_t* order;                // [2 kSrcGroups] ordered source counts and cursors
    bool fixed = false;             // the regions below are given: allocate nothing
    char* src = nullptr;            // source description
    size_t src_cap = 0;
    char* queues = nullptr;         // four queues
    size_t queue_bytes = 0;
    size_t grid_cap = 0;            // doubles the fixed grid region holds
};

RunMem ctx_mem(omc_ctx* c)
{
    return RunMem{c->d_ctrl,  c->d_counters, c->d_energies, omc::kStatsRows,
                  c->d_run,   c->d_grid,     c->d_order};
}

// Four queues of cap records each carved from a fixed region (the layout of
// ensure_queues); the counts and heads live in ctrl.
template <typename R>
void carve_queues(char* base, uint32_t cap, uint32_t* ctrl, omc::QueueView<R> q[4])
{
    char* p = base;
    auto take = [&p](size_t n) {
        char* r = p;
        p += (n + 255) & ~size_t(255);
        return r;
    };
    for (int k = 0; k < 4; ++k) {
        q[k].x = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q[k].y = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q[k].z = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q[k].u = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q[k].v = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q[k].w = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q[k].E = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q[k].vox = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q[k].hist = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q[k].qlo = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q[k].qhi = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q[k].tag = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q[k].aux_pos = reinterpret_cast<uint32_t*>(take(cap * sizeof(uint32_t)));
        q[k].aux_f = reinterpret_cast<R*>(take(cap * sizeof(R)));
        q[k].cap = cap;
        q[k].count = ctrl + 2 * k;
        q[k].head = ctrl + 2 * k + 1;
    }
}

// Kernel arguments that depend on the context only: phantom, tables, cells
// and transport parameters (the rest zero).
template <typename R>
omc::KernelArgs<R> phantom_args(const omc_ctx* c, const DeviceTables<R>& T)
{
    const omc_params& P = c->prm;
    omc::KernelArgs<R> a;
    std::memset(&a, 0, sizeof a);
    a.ph = {c->d_rho, c->d_mat, c->nx, c->ny, c->nz, R(c->dx), R(c->dy), R(c->dz),
            R(1.0 / c->dx), R(1.0 / c->dy), R(1.0 / c->dz), R(c->nx), R(c->ny), R(c->nz),
            reinterpret_cast<const uint2*>(c->d_vox)};
    const omc::EnergyGrid g = omc::energy_grid();
    a.tab.ph = T.ph;
    a.tab.muhat = T.muhat;
    a.tab.el = T.el;
    a.tab.hard = T.hard;
    a.tab.rtab = T.rtab;
    a.tab.ridx = T.ridx;
    a.tab.rshift = T.rshift;
    a.tab.rbase = T.rbase;
    a.tab.rcells = T.rcells;
    a.tab.msA = T.msA;
    a.tab.Rabs = T.Rabs;
    a.tab.n_mats = int(c->present.size());
    a.cell = {T.cellq, T.cnx, T.cny, T.cnz, T.cshift};
    a.tab.L0 = R(g.L0);
    a.tab.DL = R(g.DL);
    a.tab.INV = R(g.INV);
    a.tab.XLO = R(omc::kXLo);
    a.tab.XHI = R(omc::kXHi);
    a.tab.XINV = R(double(omc::kNA - 1) / (omc::kXHi - omc::kXLo));
    a.tab.ELo = R(omc::kELo);
    a.tab.EHi = R(omc::kEHi);
    // boundary skin (Kawrakow 2000): a voxel-limited step shorter than this is
    // taken straight to the face without the hinge deflection
    const double skin = 1e-3 * std::fmin(c->dx, std::fmin(c->dy, c->dz));
    a.prm = {R(P.Eabs_e), R(P.Eabs_g), R(P.Wcc), R(P.kc), R(P.dmax_s), R(1.0 - P.f_E), R(skin),
             P.kerma_mode, P.csda_mode};
    return a;
}

template <typename R>
int transport(omc_ctx* c, const Job& job, uint32_t seed, hipStream_t s, EventTimer& tm,
              omc_counters& L, RunMem& M)
{
    DeviceTables<R>& T = tables_of(c, R());
    int rc;
    const omc_params& P = c->prm;
    if (M.fixed) {
        // nothing may be allocated: the tables (and cell scales) must exist
        if (!T.valid || (P.photon_mode == 1 && !T.cells_valid))
            return fail(c, OMC_ESTATE, "the physics tables of this precision are not on the "
                                       "device yet: run omc_run or omc_run_device once first");
    } else {
        if ((rc = device_tables(c, T))) return rc;
        if (P.photon_mode == 1 && !T.cells_valid) {
            if ((rc = cell_scales(c, T))) return rc;
            T.cells_valid = true;
        }
    }
    const uint64_t N = job.N;
    // private copies of each tally cell (plain runs only: the beamlet
    // compaction reads one grid per cell)
    const int K = job.cell_mode ? 1 : P.tally_copies;
    const size_t need = size_t(job.cells) * size_t(K) * c->nvox;
    omc::QueueView<R> Qv[4];
    uint64_t S;
    int block, tgrid;
    if (M.fixed) {
        // one wave per CU keeps the holes of the per-wave slot reservations
        // small; the chunk is what the queue region then holds
        block = 64;
        tgrid = c->cu_count;
        const size_t per = 8 * sizeof(R) + 6 * sizeof(uint32_t);
        // a multiple of 64 records: every array of a queue 256-byte aligned
        const uint64_t cap = ((M.queue_bytes / 4) / per) & ~uint64_t(63);
        const uint64_t slack = 2 * uint64_t(tgrid) * omc::kResBlockSlots + 4096;
        const uint64_t qf = uint64_t(std::max(P.queue_factor, 1));
        if (cap <= slack || (cap - slack) / qf < 1 || cap > queue_records_max<R>())
            return fail(c, OMC_EUNSUP, "the fixed scratch holds no queue for this device");
        S = std::min<uint64_t>((cap - slack) / qf, N);
        if (P.chunk_histories > 0) S = std::min<uint64_t>(S, uint64_t(P.chunk_histories));
        if (need > M.grid_cap)
            return fail(c, OMC_EINVAL, "the tally grids (n_batches x voxels) exceed the fixed "
                                       "scratch; use fewer batches or omc_run_device");
        carve_queues<R>(M.queues, uint32_t(cap), M.ctrl, Qv);
    } else {
        DeviceQueues<R>& Q = queues_of(c, R());
        S = std::min<uint64_t>(
            P.chunk_histories > 0 ? uint64_t(P.chunk_histories) : (uint64_t(1) << 24), N);
        block = P.block_size;
        tgrid = c->cu_count * P.blocks_per_cu;
        // capacity: secondaries per source history, plus the holes left by the
        // per-wave slot reservations of the two kernels that append to a queue;
        // a chunk too large for the largest queue is cut down to fit
        const uint64_t waves = uint64_t(tgrid) * (block / 64);
        const uint64_t slack = 2 * waves * omc::kResBlockSlots + 4096;
        const uint64_t qmax = queue_records_max<R>();
        const uint64_t qf = uint64_t(std::max(P.queue_factor, 1));
        if (qmax <= slack + qf) return fail(c, OMC_EUNSUP, "launch shape too large for the queues");
        S = std::min<uint64_t>(S, (qmax - slack) / qf);
        const uint64_t qcap = qf * S + slack;
        if ((rc = ensure_queues(c, Q, uint32_t(std::max<uint64_t>(qcap, S)), uint32_t(qcap))))
            return rc;
        for (int k = 0; k < 4; ++k) Qv[k] = Q.q[k];
        if (c->grid_cells < size_t(job.cells) * size_t(K)) {
            drop_graph(c);
            dfree(c->d_grid);
            c->grid_cells = 0;
            if (hipMalloc(&c->d_grid, need * sizeof(double)) != hipSuccess) {
                c->d_grid = nullptr;
                return fail(c, OMC_ENOMEM, "hipMalloc failed for the tally grids");
            }
            c->grid_cells = size_t(job.cells) * size_t(K);
        }
        M.grid = c->d_grid;
    }
    // launch checks read the runtime's last error: start from a clean state
    (void)hipGetLastError();
    omc::SourceView<R> sv{};
    if ((rc = pack_sources(c, job, s, sv, M.fixed ? M.src : nullptr, M.src_cap))) return rc;
    c->h_run->seed = seed;
    c->h_run->n_batches = job.cell_mode ? 0u : uint32_t(job.cells);
    c->h_run->n_total = N;
    HIP_TRY(c, hipMemcpyAsync(M.run, c->h_run, sizeof(omc::RunDesc), hipMemcpyHostToDevice, s));

    omc::KernelArgs<R> a = phantom_args(c, T);
    a.tally = {M.grid, c->nvox, uint32_t(K - 1)};
    a.stats = {M.counters, M.energies, M.rows, M.ctrl + 8, M.ctrl + 9, M.ctrl + 10};
    a.src = sv;
    a.trace = c->trace;
    a.run = M.run;
    a.chunk = 64;
    a.min_grid = c->cu_count;
    a.spill_lanes = P.straggler_lanes;
    a.event_lanes = P.event_lanes;
    // the ordered source (Sec. 2.2.1: energy bin by energy bin) where the
    // particles' energies differ: a spectrum or a phase space
    bool spread = false;
    for (const HostBeam& hb : job.beams)
        spread = spread || hb.src.geometry == 2 || hb.src.n_bins > 0;
    a.src_order = P.source_order == 1 && spread ? M.order : nullptr;

    const int nm = int(c->present.size());
    int lds_max = 0, lds_cu = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    HIP_TRY(c, hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                     c->device));
    // per-material tables in LDS while two work-groups of each kernel still fit
    // a CU with them; else read from global memory (through L2). On MI355X, 8
    // materials (66 KB in FP32, two work-groups) run faster from LDS at 4 to 8
    // requested work-groups per CU, 16 (130 KB, one work-group) from global
    const size_t lds_tabs = std::max(omc::photon_lds_bytes<R>(nm), omc::electron_lds_bytes<R>(nm));
    const bool gtab = P.table_mode == 2 || (P.table_mode == 0 && 2 * lds_tabs > size_t(lds_cu));
    const bool cells = P.photon_mode == 1;
    const size_t lds_ph =
        omc::photon_lds_bytes<R>(nm, gtab, cells ? T.cnx * T.cny * T.cnz : 0);
    const size_t lds_el = omc::electron_lds_bytes<R>(nm, gtab);
    if (lds_ph > size_t(lds_max) || lds_el > size_t(lds_max))
        return fail(c, OMC_EUNSUP, "material tables exceed the LDS of a work-group; use "
                                   "table_mode 0 or 2 (tables in global memory)");
    if (omc::Launch<R>::prepare(lds_ph, lds_el, gtab))
        return fail(c, OMC_EDEVICE, "cannot raise the LDS limit of the transport kernels");
    c->last_gtab = gtab;
    c->timing.tables_global = gtab ? 1 : 0;

    auto zero_all = [&](hipStream_t st) {
        return omc::launch_zero(M.grid, need, st) ||
               omc::launch_zero(M.counters, size_t(M.rows) * omc::kNumCounters, st) ||
               omc::launch_zero(M.energies, size_t(M.rows) * omc::kNumEnergies, st) ||
               omc::launch_zero(M.ctrl, 8, st) ||
               omc::launch_zero(M.order, omc::kSrcGroups, st);
    };
    auto source = [&](uint64_t begin, uint32_t cnt, int pc, int ec, hipStream_t st,
                      EventTimer& t) {
        a.qp_out = Qv[pc];
        a.qe_out = Qv[ec];
        a.src_begin = begin;
        a.src_count = cnt;
        t.begin(0);
        const uint32_t per = a.src_order ? 256u * omc::kSrcOrderItems : 256u;
        const int grid = int((uint64_t(cnt) + per - 1) / per);
        const int e = (a.src_order && (omc::Launch<R>::source_groups(a, grid, st) ||
                                       omc::launch_source_scan(M.order, st))) ||
                      omc::Launch<R>::source(a, grid, 256, st);
        t.end();
        return e || omc::launch_queue_commit(M.ctrl, job.particle == 0 ? pc : ec, cnt, st);
    };
    auto generation = [&](int pc, int ec, bool photons, hipStream_t st, EventTimer& t) {
        int e = 0;
        if (photons) {
            a.qin = Qv[pc];
            a.qe_out = Qv[ec];
            a.qp_out = Qv[pc ^ 1];
            t.begin(1);
            e = omc::Launch<R>::photon(a, tgrid, block, lds_ph, gtab, cells, st);
            t.end();
        }
        a.qin = Qv[ec];
        a.qe_out = Qv[ec ^ 1];
        a.qp_out = Qv[pc ^ 1];
        t.begin(2);
        e = e || omc::Launch<R>::electron(a, tgrid, block, lds_el, P.electron_mode == 1, gtab,
                                          st);
        t.end();
        return e || omc::launch_queue_reset(M.ctrl, (1 << pc) | (1 << ec), st);
    };
    uint32_t iters = 0;
    auto readback = [&](int pc, int ec, uint32_t& n_ph, uint32_t& n_el) -> int {
        HIP_TRY(c, hipMemcpyAsync(c->h_ctrl, M.ctrl, 16 * sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        if (c->h_ctrl[8])
            return fail(c, OMC_EQUEUE,
                        "secondary particle queue overflow; raise queue_factor or lower "
                        "chunk_histories");
        n_ph = c->h_ctrl[2 * pc];
        n_el = c->h_ctrl[2 * ec];
        return OMC_OK;
    };
    // host-driven generations until both queues are empty
    auto drain = [&](int& pc, int& ec, uint32_t n_ph, uint32_t n_el) -> int {
        while (n_ph || n_el) {
            if (++iters > 100000) return fail(c, OMC_ENUMERIC, "generation limit exceeded");
            if (generation(pc, ec, n_ph != 0, s, tm))
                return fail(c, OMC_EDEVICE, "transport kernel launch failed");
            pc ^= 1;
            ec ^= 1;
            const int e = readback(pc, ec, n_ph, n_el);
            if (e) return e;
        }
        return OMC_OK;
    };

    int pc = 0, ec = 2;  // current photon / electron queues
    if (!M.fixed && P.graph_depth > 0 && P.timing) {
        // HIP events do not time kernels inside a graph: the timed variant
        // launches the same fixed-depth sequence eagerly, one event pair per
        // launch (same kernels, same grids, same carry-over)
        if (zero_all(s)) return fail(c, OMC_EDEVICE, "zero-fill launch failed");
        for (uint64_t done = 0; done < N; done += S) {
            const uint32_t cnt = uint32_t(std::min<uint64_t>(S, N - done));
            if (source(done, cnt, pc, ec, s, tm))
                return fail(c, OMC_EDEVICE, "source kernel launch failed");
            for (int k = 0; k < P.graph_depth; ++k, ++iters) {
                if (generation(pc, ec, true, s, tm))
                    return fail(c, OMC_EDEVICE, "transport kernel launch failed");
                pc ^= 1;
                ec ^= 1;
            }
        }
        uint32_t n_ph = 0, n_el = 0;
        if ((rc = readback(pc, ec, n_ph, n_el))) return rc;
        if ((rc = drain(pc, ec, n_ph, n_el))) return rc;
    } else if (M.fixed || P.graph_depth <= 0) {
        if (zero_all(s)) return fail(c, OMC_EDEVICE, "zero-fill launch failed");
        for (uint64_t done = 0; done < N; done += S) {
            const uint32_t cnt = uint32_t(std::min<uint64_t>(S, N - done));
            if (source(done, cnt, pc, ec, s, tm))
                return fail(c, OMC_EDEVICE, "source kernel launch failed");
            // the queues were drained before this chunk
            if ((rc = drain(pc, ec, job.particle == 0 ? cnt : 0, job.particle == 0 ? 0 : cnt)))
                return rc;
        }
    } else {
        const int K = P.graph_depth;
        // everything the captured launches depend on; a change means a new capture
        std::vector<unsigned char> key(sizeof a + 16 * sizeof(uint64_t));
        const uint64_t shape[16] = {sizeof(R), N,      S,      uint64_t(K), uint64_t(block),
                                    uint64_t(tgrid),   lds_ph, lds_el,      uint64_t(P.timing),
                                    uint64_t(job.particle), need, uint64_t(P.electron_mode),
                                    uint64_t(gtab), uint64_t(P.photon_mode), 0, 0};
        std::memcpy(key.data(), &a, sizeof a);
        std::memcpy(key.data() + sizeof a, shape, sizeof shape);
        if (!c->graph || key != c->graph_key) {
            drop_graph(c);
            if (!c->cap_stream &&
                hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
                c->cap_stream = nullptr;
                return fail(c, OMC_EDEVICE, "cannot create the capture stream");
            }
            EventTimer gt;  // not recording: events cannot time kernels inside a graph
            gt.s = c->cap_stream;
            HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            int e = zero_all(c->cap_stream);
            int gpc = 0, gec = 2;
            uint32_t giters = 0;
            for (uint64_t done = 0; done < N && !e; done += S) {
                const uint32_t cnt = uint32_t(std::min<uint64_t>(S, N - done));
                e = source(done, cnt, gpc, gec, c->cap_stream, gt);
                for (int k = 0; k < K && !e; ++k) {
                    e = generation(gpc, gec, true, c->cap_stream, gt);
                    gpc ^= 1;
                    gec ^= 1;
                    ++giters;
                }
            }
            hipGraph_t gr = nullptr;
            const hipError_t ce = hipStreamEndCapture(c->cap_stream, &gr);
            hipGraphExec_t ex = nullptr;
            const hipError_t ie = (e || ce != hipSuccess || !gr)
                                      ? hipErrorUnknown
                                      : hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            if (gr) (void)hipGraphDestroy(gr);
            if (e || ce != hipSuccess || ie != hipSuccess) {
                (void)hipGetLastError();
                return fail(c, OMC_EDEVICE, std::string("graph capture failed: ") +
                                                hipGetErrorString(ce != hipSuccess ? ce : ie));
            }
            c->graph = ex;
            c->graph_key = key;
            c->graph_pc = gpc;
            c->graph_ec = gec;
            c->graph_iters = giters;
        }
        HIP_TRY(c, hipGraphLaunch(c->graph, s));
        iters += c->graph_iters;
        pc = c->graph_pc;
        ec = c->graph_ec;
        uint32_t n_ph = 0, n_el = 0;
        if ((rc = readback(pc, ec, n_ph, n_el))) return rc;
        if ((rc = drain(pc, ec, n_ph, n_el))) return rc;
    }
    L.iterations += iters;
    return OMC_OK;
}

// Sum the per-work-group statistics and read them (and the control words)
// into L; accumulate adds to what L holds.
int finish_stats(omc_ctx* c, hipStream_t s, omc_counters& L, bool accumulate, const RunMem& M)
{
    unsigned long long cnts[omc::kNumCounters];
    double en[omc::kNumEnergies];
    if (omc::launch_stats_reduce(M.counters, M.energies, M.rows, s))
        return fail(c, OMC_EDEVICE, "statistics reduce launch failed");
    HIP_TRY(c, hipMemcpyAsync(c->h_ctrl, M.ctrl, 16 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(cnts, M.counters, sizeof cnts, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(en, M.energies, sizeof en, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (!accumulate) {
        const uint32_t it = L.iterations;
        L = omc_counters{};
        L.iterations = it;
    }
    for (int k = 0; k < omc::kNumCounters; ++k) L.*kCounterField[k] += cnts[k];
    L.E_incident += en[omc::EN_INCIDENT];
    L.E_deposited += en[omc::EN_DEPOSITED];
    L.E_escaped += en[omc::EN_ESCAPED];
    L.E_pair_rest = double(L.ph_pair) * 2.0 * omc::kMC2;
    L.E_annih_rest = double(L.pos_annihil) * 2.0 * omc::kMC2;
    L.max_steps = std::max(L.max_steps, c->h_ctrl[9]);
    L.queue_hwm_el = std::max<uint64_t>(L.queue_hwm_el, c->h_ctrl[10]);
    L.queue_hwm_ph = std::max<uint64_t>(L.queue_hwm_ph, c->h_ctrl[11]);
    return OMC_OK;
}

int check_ledger(omc_ctx* c, const omc_counters& L)
{
    const double lhs = L.E_incident + L.E_annih_rest - L.E_pair_rest;
    const double rhs = L.E_deposited + L.E_escaped;
    if (!std::isfinite(lhs) || !std::isfinite(rhs) || std::fabs(lhs - rhs) > 1e-9 * std::fabs(lhs))
        return fail(c, OMC_ENUMERIC, "energy ledger violated: incident+annihilation-pair != "
                                     "deposited+escaped");
    return OMC_OK;
}

template <typename R>
int run_impl(omc_ctx* c, uint64_t N, uint32_t seed, uint32_t h0, double* d_dose, double* d_dose2,
             hipStream_t s, RunMem* fixed = nullptr)
{
    RunMem M = fixed ? *fixed : ctx_mem(c);
    const omc_params& P = c->prm;
    Job job;
    job.beams.push_back(HostBeam{c->src, &c->edges, &c->cdf, N, h0, &c->psf, c->psf_dev});
    job.particle = c->src.particle;
    job.cell_mode = 0;
    job.cells = P.n_batches;
    job.N = N;
    c->timing = omc_timing{};
    EventTimer tm;
    tm.on = P.timing != 0 && !M.fixed;
    tm.s = s;
    RunClock clk;
    clk.start(tm.on, s);
    omc_counters& L = c->last;
    L = omc_counters{};
    int rc = transport<R>(c, job, seed, s, tm, L, M);
    if (rc == OMC_OK) {
        std::vector<double> nb;
        batch_sizes(N, job.cells, nb);
        tm.begin(3);
        if (omc::launch_fold(M.grid, c->d_rho, c->nvox, job.cells, P.tally_copies, nb.data(),
                             c->dx * c->dy * c->dz, double(N), d_dose, d_dose2, s))
            rc = fail(c, OMC_EDEVICE, "fold kernel launch failed");
        tm.end();
        clk.stop(s);
        if (rc == OMC_OK) rc = finish_stats(c, s, L, false, M);
    }
    (void)hipStreamSynchronize(s);
    collect_events(tm.ev, c->timing);
    destroy_events(tm.ev);
    clk.collect(c->timing);
    if (rc) return rc;
    return check_ledger(c, L);
}

// ------------------------------------------------------------------ beamlets
struct SparsePart {
    uint32_t* voxel = nullptr;
    float* dose = nullptr;
    uint64_t nnz = 0;
};

void free_parts(std::vector<SparsePart>& parts)
{
    for (auto& p : parts) {
        dfree(p.voxel);
        dfree(p.dose);
    }
    parts.clear();
}

int ensure_cscratch(omc_ctx* c, size_t bytes)
{
    if (c->cscratch_cap >= bytes) return OMC_OK;
    dfree(c->d_cscratch);
    c->cscratch_cap = 0;
    if (hipMalloc(&c->d_cscratch, bytes) != hipSuccess) {
        c->d_cscratch = nullptr;
        return fail(c, OMC_ENOMEM, "hipMalloc failed for the compaction scratch");
    }
    c->cscratch_cap = bytes;
    return OMC_OK;
}

// Compact the cell grids of one group of beams into device CSR arrays; rows
// receives the group's n_beams + 1 row offsets (starting at 0).
int compact_group(omc_ctx* c, const Job& job, hipStream_t s, EventTimer& tm, SparsePart& part,
                  std::vector<uint64_t>& rows)
{
    const int G = job.cells;
    const size_t tiles = (c->nvox + omc::kCompactTile - 1) / omc::kCompactTile;
    const size_t nt = size_t(G) * tiles;
    const size_t n_seg = (nt + 1023) / 1024;
    const size_t o_scale = 0;
    const size_t o_thr = o_scale + align256(size_t(G) * sizeof(double));
    const size_t o_cnt = o_thr + align256(size_t(G) * sizeof(float));
    const size_t o_off = o_cnt + align256(nt * sizeof(uint32_t));
    const size_t o_tmp = o_off + align256((nt + 1) * sizeof(uint64_t));
    const size_t bytes = o_tmp + align256((n_seg + 1) * sizeof(uint64_t));
    int rc = ensure_cscratch(c, bytes);
    if (rc) return rc;
    double* d_scale = reinterpret_cast<double*>(c->d_cscratch + o_scale);
    float* d_thr = reinterpret_cast<float*>(c->d_cscratch + o_thr);
    uint32_t* d_cnt = reinterpret_cast<uint32_t*>(c->d_cscratch + o_cnt);
    uint64_t* d_off = reinterpret_cast<uint64_t*>(c->d_cscratch + o_off);
    uint64_t* d_tmp = reinterpret_cast<uint64_t*>(c->d_cscratch + o_tmp);

    const double V = c->dx * c->dy * c->dz;
    std::vector<double> scale(G);
    for (int b = 0; b < G; ++b) scale[b] = 1.0 / (V * double(job.beams[b].n));
    HIP_TRY(c, hipMemcpyAsync(d_scale, scale.data(), G * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemsetAsync(d_thr, 0, G * sizeof(float), s));
    const double thr_rel = c->prm.sparse_threshold;
    std::vector<float> mx(G);  // host memory of an asynchronous copy: alive until the sync below
    tm.begin(3);
    if (thr_rel > 0) {
        if (omc::launch_beam_max(c->d_grid, c->d_rho, c->nvox, G, d_scale, d_thr, s))
            return fail(c, OMC_EDEVICE, "beam maximum launch failed");
        HIP_TRY(c, hipMemcpyAsync(mx.data(), d_thr, G * sizeof(float), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        for (float& m : mx) m = float(double(m) * thr_rel);
        HIP_TRY(c, hipMemcpyAsync(d_thr, mx.data(), G * sizeof(float), hipMemcpyHostToDevice, s));
    }
    if (omc::launch_compact_count(c->d_grid, c->d_rho, c->nvox, G, d_scale, d_thr, d_cnt, s) ||
        omc::launch_scan(d_cnt, d_off, nt, d_tmp, s))
        return fail(c, OMC_EDEVICE, "compaction count/scan launch failed");
    tm.end();
    // row b starts at the offset of its first tile; the last row ends at the total
    rows.assign(size_t(G) + 1, 0);
    HIP_TRY(c, hipMemcpy2DAsync(rows.data(), sizeof(uint64_t), d_off, tiles * sizeof(uint64_t),
                                sizeof(uint64_t), size_t(G) + 1, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    part.nnz = rows[G];
    if (part.nnz == 0) return OMC_OK;
    if (hipMalloc(&part.voxel, part.nnz * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&part.dose, part.nnz * sizeof(float)) != hipSuccess) {
        dfree(part.voxel);
        dfree(part.dose);
        return fail(c, OMC_ENOMEM, "hipMalloc failed for the sparse dose rows");
    }
    tm.begin(3);
    if (omc::launch_compact_write(c->d_grid, c->d_rho, c->nvox, G, d_scale, d_thr, d_off,
                                  part.nnz, part.voxel, part.dose, s))
        return fail(c, OMC_EDEVICE, "compaction write launch failed");
    tm.end();
    return OMC_OK;
}

template <typename R>
int beamlets_impl(omc_ctx* c, const std::vector<HostBeam>& beams, int particle, uint32_t seed,
                  int on_device, hipStream_t s, omc_sparse_out* out)
{
    const omc_params& P = c->prm;
    const int n = int(beams.size());
    const size_t tiles = (c->nvox + omc::kCompactTile - 1) / omc::kCompactTile;
    int G = P.beamlet_group > 0 ? std::min(P.beamlet_group, n) : 0;
    if (G == 0) {
        size_t freeb = 0, totalb = 0;
        HIP_TRY(c, hipMemGetInfo(&freeb, &totalb));
        const size_t per = c->nvox * sizeof(double);
        const size_t budget = freeb / 2 + c->grid_cells * per;
        G = int(std::max<size_t>(1, std::min<size_t>(size_t(n), budget / per)));
    }
    // cell ids fit the 24 bits of a record tag, the compaction grid and the scan
    G = std::min(G, 65535);
    while (G > 1 && size_t(G) * tiles > (size_t(1) << 31)) G /= 2;

    c->timing = omc_timing{};
    EventTimer tm;
    tm.on = P.timing != 0;
    tm.s = s;
    RunClock clk;
    clk.start(tm.on, s);
    omc_counters& L = c->last;
    L = omc_counters{};
    std::vector<SparsePart> parts;
    std::vector<uint64_t> rows(size_t(n) + 1, 0);
    int rc = OMC_OK;
    for (int g0 = 0; g0 < n && rc == OMC_OK; g0 += G) {
        const int gn = std::min(G, n - g0);
        Job job;
        job.beams.assign(beams.begin() + g0, beams.begin() + g0 + gn);
        job.particle = particle;
        job.cell_mode = 1;
        job.cells = gn;
        for (const auto& b : job.beams) job.N += b.n;
        RunMem M = ctx_mem(c);
        rc = transport<R>(c, job, seed, s, tm, L, M);
        SparsePart part;
        std::vector<uint64_t> grows;
        if (rc == OMC_OK) rc = compact_group(c, job, s, tm, part, grows);
        if (rc == OMC_OK) rc = finish_stats(c, s, L, g0 > 0, M);
        if (rc == OMC_OK) {
            const uint64_t base = rows[g0];
            for (int b = 0; b < gn; ++b) rows[g0 + b + 1] = base + grows[b + 1];
        }
        parts.push_back(part);
    }
    clk.stop(s);
    (void)hipStreamSynchronize(s);
    collect_events(tm.ev, c->timing);
    destroy_events(tm.ev);
    clk.collect(c->timing);
    if (rc == OMC_OK) rc = check_ledger(c, L);
    if (rc) {
        free_parts(parts);
        return rc;
    }
    // assemble the rows of all groups
    const uint64_t nnz = rows[n];
    out->n_beamlets = n;
    out->on_device = on_device;
    out->nnz = nnz;
    out->row_ptr = static_cast<uint64_t*>(std::malloc((size_t(n) + 1) * sizeof(uint64_t)));
    if (!out->row_ptr) {
        free_parts(parts);
        return fail(c, OMC_ENOMEM, "host allocation failed for the row offsets");
    }
    std::memcpy(out->row_ptr, rows.data(), (size_t(n) + 1) * sizeof(uint64_t));
    if (nnz == 0) {
        free_parts(parts);
        return OMC_OK;
    }
    if (on_device && parts.size() == 1) {
        out->voxel = parts[0].voxel;
        out->dose = parts[0].dose;
        parts[0] = SparsePart{};
        return OMC_OK;
    }
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (on_device) {
        if (hipMalloc(&out->voxel, nnz * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(&out->dose, nnz * sizeof(float)) != hipSuccess)
            rc = fail(c, OMC_ENOMEM, "hipMalloc failed for the sparse dose rows");
    } else {
        out->voxel = static_cast<uint32_t*>(std::malloc(nnz * sizeof(uint32_t)));
        out->dose = static_cast<float*>(std::malloc(nnz * sizeof(float)));
        if (!out->voxel || !out->dose)
            rc = fail(c, OMC_ENOMEM, "host allocation failed for the sparse dose rows");
    }
    uint64_t at = 0;
    for (const auto& p : parts) {
        if (rc || p.nnz == 0) continue;
        if (hipMemcpyAsync(out->voxel + at, p.voxel, p.nnz * sizeof(uint32_t), kind, s) !=
                hipSuccess ||
            hipMemcpyAsync(out->dose + at, p.dose, p.nnz * sizeof(float), kind, s) != hipSuccess)
            rc = fail(c, OMC_EDEVICE, "copy of the sparse dose rows failed");
        at += p.nnz;
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == OMC_OK)
        rc = fail(c, OMC_EDEVICE, "copy of the sparse dose rows failed");
    free_parts(parts);
    return rc;
}

}  // namespace

namespace {

// omc_debug_sample for one transport precision: the samples run on the
// device in a scratch block of their own (queues for the products, control
// words, statistics, a one-cell tally, the records), released at the end.
template <typename R>
int debug_sample_impl(omc_ctx* c, int which, const double* args, uint32_t seed, uint32_t n,
                      double* out, uint32_t* words)
{
    DeviceTables<R>& T = tables_of(c, R());
    int rc = device_tables(c, T);
    if (rc) return rc;
    const uint64_t waves = (uint64_t(n) + 63) / 64;
    const uint32_t cap = uint32_t(((2 * uint64_t(n) + 128 * waves + 256) + 63) & ~uint64_t(63));
    const size_t per = 8 * sizeof(R) + 6 * sizeof(uint32_t);
    const size_t qbytes = size_t(cap) * per;
    const size_t bytes = 2 * qbytes + 256 + 256 + 8 * 64 + align256(size_t(n) * omc::kSampleWords *
                         sizeof(double)) + align256(size_t(n) * sizeof(uint32_t));
    char* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess)
        return fail(c, OMC_ENOMEM, "hipMalloc failed for the sampler");
    char* p = mem;
    auto take = [&p](size_t k) {
        char* r = p;
        p += (k + 255) & ~size_t(255);
        return r;
    };
    omc::QueueView<R> q[2];
    uint32_t* ctrl = nullptr;
    char* qmem[2] = {take(qbytes), take(qbytes)};
    ctrl = reinterpret_cast<uint32_t*>(take(16 * sizeof(uint32_t)));
    auto* counters = reinterpret_cast<unsigned long long*>(take(omc::kNumCounters * 8));
    auto* energies = reinterpret_cast<double*>(take(omc::kNumEnergies * 8 + 8 * 8));
    double* tally = energies + 8;
    double* d_out = reinterpret_cast<double*>(take(size_t(n) * omc::kSampleWords * sizeof(double)));
    uint32_t* d_words = reinterpret_cast<uint32_t*>(take(size_t(n) * sizeof(uint32_t)));
    for (int k = 0; k < 2; ++k) {
        char* b = qmem[k];
        auto arr = [&b, cap](size_t elem) {
            char* r = b;
            b += size_t(cap) * elem;
            return r;
        };
        q[k].x = reinterpret_cast<R*>(arr(sizeof(R)));
        q[k].y = reinterpret_cast<R*>(arr(sizeof(R)));
        q[k].z = reinterpret_cast<R*>(arr(sizeof(R)));
        q[k].u = reinterpret_cast<R*>(arr(sizeof(R)));
        q[k].v = reinterpret_cast<R*>(arr(sizeof(R)));
        q[k].w = reinterpret_cast<R*>(arr(sizeof(R)));
        q[k].E = reinterpret_cast<R*>(arr(sizeof(R)));
        q[k].vox = reinterpret_cast<uint32_t*>(arr(4));
        q[k].hist = reinterpret_cast<uint32_t*>(arr(4));
        q[k].qlo = reinterpret_cast<uint32_t*>(arr(4));
        q[k].qhi = reinterpret_cast<uint32_t*>(arr(4));
        q[k].tag = reinterpret_cast<uint32_t*>(arr(4));
        q[k].aux_pos = reinterpret_cast<uint32_t*>(arr(4));
        q[k].aux_f = reinterpret_cast<R*>(arr(sizeof(R)));
        q[k].cap = cap;
        q[k].count = ctrl + 2 * k;
        q[k].head = ctrl + 2 * k + 1;
    }
    auto bail = [&](int code, const std::string& msg) {
        (void)hipGetLastError();
        (void)hipFree(mem);
        return fail(c, code, msg);
    };
    if (hipMemset(ctrl, 0, 16 * sizeof(uint32_t)) != hipSuccess ||
        hipMemset(counters, 0, omc::kNumCounters * 8) != hipSuccess ||
        hipMemset(energies, 0, (omc::kNumEnergies + 8) * 8) != hipSuccess ||
        hipMemset(d_out, 0, size_t(n) * omc::kSampleWords * sizeof(double)) != hipSuccess)
        return bail(OMC_EDEVICE, "hipMemset failed for the sampler");
    omc::KernelArgs<R> a = phantom_args(c, T);
    // every product is kept
    a.prm.Eabs_e = R(0);
    a.prm.Eabs_g = R(0);
    a.prm.kerma = 0;
    a.tally = {tally, c->nvox, 0u};
    a.stats = {counters, energies, 1u, ctrl + 8, ctrl + 9, ctrl + 10};
    a.qe_out = q[0];
    a.qp_out = q[1];
    int e = 0;
    if (which == omc::SMP_SOURCE) {
        Job job;
        job.beams.push_back(HostBeam{c->src, &c->edges, &c->cdf, n, 0u, &c->psf, c->psf_dev});
        job.particle = c->src.particle;
        job.cells = 1;
        job.N = n;
        omc::SourceView<R> sv{};
        if ((rc = pack_sources(c, job, nullptr, sv))) {
            (void)hipFree(mem);
            return rc;
        }
        c->h_run->seed = seed;
        c->h_run->n_batches = 1;
        c->h_run->n_total = n;
        if (hipMemcpy(c->d_run, c->h_run, sizeof(omc::RunDesc), hipMemcpyHostToDevice) !=
            hipSuccess)
            return bail(OMC_EDEVICE, "run descriptor upload failed");
        a.src = sv;
        a.run = c->d_run;
        a.src_begin = 0;
        a.src_count = n;
        e = omc::Launch<R>::source(a, int((n + 255) / 256), 256, nullptr);
    } else {
        omc::SampleArgs sa{which, seed, n, args[0], args[1], args[2], args[3], args[4]};
        e = omc::Launch<R>::sample(a, sa, d_out, d_words, nullptr);
    }
    if (e || hipDeviceSynchronize() != hipSuccess) return bail(OMC_EDEVICE, "sampler launch failed");
    uint32_t h_ctrl[16];
    if (hipMemcpy(h_ctrl, ctrl, sizeof h_ctrl, hipMemcpyDeviceToHost) != hipSuccess)
        return bail(OMC_EDEVICE, "sampler readback failed");
    if (h_ctrl[8]) return bail(OMC_EQUEUE, "sampler product queue overflow");
    if (which != omc::SMP_SOURCE &&
        (hipMemcpy(out, d_out, size_t(n) * omc::kSampleWords * sizeof(double),
                   hipMemcpyDeviceToHost) != hipSuccess ||
         hipMemcpy(words, d_words, size_t(n) * sizeof(uint32_t), hipMemcpyDeviceToHost) !=
             hipSuccess))
        return bail(OMC_EDEVICE, "sampler readback failed");
    // the products (or, for the source, the entering particles) from the queues.
    // The source kernel writes history k to slot k of its particle's queue (a
    // hole for a ray that misses the phantom) and leaves the count to the
    // commit kernel of a run, which the sampler does not launch.
    if (which == omc::SMP_SOURCE) std::memset(out, 0, size_t(n) * omc::kSampleWords * sizeof(double));
    const int src_q = c->src.particle == 0 ? 1 : 0;
    for (int k = 0; k < 2; ++k) {
        const uint32_t cnt =
            which == omc::SMP_SOURCE ? (k == src_q ? n : 0u) : std::min(h_ctrl[2 * k], cap);
        if (cnt == 0) continue;
        std::vector<R> E(cnt), u(cnt), v(cnt), w(cnt), x(cnt), y(cnt), z(cnt);
        std::vector<uint32_t> hist(cnt), tag(cnt);
        const std::pair<const void*, void*> cp[] = {
            {q[k].E, E.data()}, {q[k].u, u.data()}, {q[k].v, v.data()}, {q[k].w, w.data()},
            {q[k].x, x.data()}, {q[k].y, y.data()}, {q[k].z, z.data()}};
        for (const auto& pr : cp)
            if (hipMemcpy(pr.second, pr.first, cnt * sizeof(R), hipMemcpyDeviceToHost) !=
                hipSuccess)
                return bail(OMC_EDEVICE, "sampler readback failed");
        if (hipMemcpy(hist.data(), q[k].hist, cnt * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(tag.data(), q[k].tag, cnt * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return bail(OMC_EDEVICE, "sampler readback failed");
        for (uint32_t i = 0; i < cnt; ++i) {
            if (tag[i] == omc::kHoleTag) continue;
            if (which == omc::SMP_SOURCE) {
                if (i >= n) continue;
                double* r = out + size_t(omc::kSampleWords) * i;
                r[0] = double(E[i]);
                r[1] = double(u[i]);
                r[2] = double(v[i]);
                r[3] = double(w[i]);
                r[5] = double(x[i]);
                r[6] = double(y[i]);
                r[7] = double(z[i]);
                r[15] = 1.0;
                continue;
            }
            const uint32_t h = hist[i];
            if (h >= n) continue;
            double* r = out + size_t(omc::kSampleWords) * h;
            const int j = int(r[4]);
            r[4] = double(j + 1);
            if (j >= 2) continue;
            r[5 + 4 * j] = double(E[i]);
            r[6 + 4 * j] = double(u[i]);
            r[7 + 4 * j] = double(v[i]);
            r[8 + 4 * j] = double(w[i]);
            r[13 + j] = double(tag[i] & 0x7Fu);
        }
    }
    if (which == omc::SMP_SOURCE) {
        for (uint32_t i = 0; i < n; ++i) words[i] = 4u;
    } else if (which == omc::SMP_PAIR) {
        const double K = args[0] - 2.0 * omc::kMC2;
        for (uint32_t i = 0; i < n; ++i) {
            double* r = out + size_t(omc::kSampleWords) * i;
            r[15] = r[4] > 0 ? r[5] / K : 0.0;
        }
    }
    (void)hipFree(mem);
    return OMC_OK;
}

}  // namespace

// ------------------------------------------------------ fixed device scratch
// omc_run_device_static runs without allocating device memory: its queues,
// tally grids, statistics, control words and source description are regions
// of one file-scope device array. Every GPU the library runs on holds its own
// copy from module load until the process ends. In host code the array's name
// is a host-side stand-in, not a device address: the address of each GPU's
// copy is looked up once per device with hipGetSymbolAddress (at the first
// omc_create on that device, with the device current), and only that address
// is passed to kernels and copies.
namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr uint32_t kScratchRows = 64;  // statistics rows (work-groups share them by index)
constexpr size_t kScrCtrl = 0;         // 64 control words
constexpr size_t kScrRun = 256;        // run descriptor
constexpr size_t kScrOrder = 512;      // ordered source counts and cursors
constexpr size_t kScrCounters = 1024;
static_assert(kScrOrder + 2 * omc::kSrcGroups * sizeof(uint32_t) <= kScrCounters, "layout");
constexpr size_t kScrEnergies =
    kScrCounters + ((size_t(kScratchRows) * omc::kNumCounters * 8 + 255) & ~size_t(255));
constexpr size_t kScrSrc =
    kScrEnergies + ((size_t(kScratchRows) * omc::kNumEnergies * 8 + 255) & ~size_t(255));
constexpr size_t kScrSrcBytes = size_t(1) << 20;   // beams, history prefix, spectra
constexpr size_t kScrGrid = (kScrSrc + kScrSrcBytes + 255) & ~size_t(255);
constexpr size_t kScrGridBytes = size_t(48) << 20;  // tally cells: 6291456 doubles
constexpr size_t kScrQueues = kScrGrid + kScrGridBytes;
constexpr size_t kScrQueueBytes = kScratchBytes - kScrQueues;  // the four particle queues
static_assert(kScrQueues % 256 == 0 && kScrQueueBytes > (size_t(64) << 20), "scratch layout");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kScratchDevices] = {};
bool g_scratch_seen[kScratchDevices] = {};

// The device address of the current device's copy of the scratch array
// (NULL if the lookup failed); looked up once per device.
char* scratch_of_device(int device)
{
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_seen[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[device] = e == hipSuccess ? static_cast<char*>(p) : nullptr;
        g_scratch_seen[device] = true;
        (void)hipGetLastError();
    }
    return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

void omc_default_params(omc_params* p)
{
    if (!p) return;
    *p = omc_params{};
    p->Eabs_e = 0.2;
    p->Eabs_g = 0.05;
    p->Wcc = 0.05;
    p->kc = 0.2;
    p->dmax_s = 0.5;
    p->f_E = 0.25;
    p->n_batches = 10;
    p->parity_fp64 = 0;
    p->kerma_mode = 0;
    p->csda_mode = 0;
    p->block_size = 256;
    p->blocks_per_cu = 4;
    p->chunk_histories = 0;
    p->queue_factor = 6;
    p->timing = 0;
    p->graph_depth = 0;
    p->beamlet_group = 0;
    p->sparse_threshold = 0.0;
    p->straggler_lanes = 16;
    p->electron_mode = 0;
    p->table_mode = 0;
    p->photon_mode = 0;
    p->tally_copies = 1;
    p->source_order = 0;
    p->event_lanes = 12;
}

int check_phantom(const float* density, const uint8_t* material, size_t nvox, int n_mats,
                  std::vector<double>& rmax);
int upload_phantom(omc_ctx* c, const float* density, const uint8_t* material);

// The built-in library (mats == NULL in omc_create): 0 water, 1 lung, 2
// cortical bone, the three materials of the paper's slab and half-slab
// phantoms (Sec. 2.2 "Materials"). Mass fractions (normalised), atomic
// weights in g/mol, I in eV and the nominal density of each; the
// compositions are ICRU-44-like input data.
namespace {
const int kBiZ0[] = {1, 8};
const double kBiA0[] = {1.008, 15.999};
const double kBiW0[] = {0.111894, 0.888106};
const int kBiZ1[] = {1, 6, 7, 8, 11, 15, 16, 17, 19};
const double kBiA1[] = {1.008, 12.011, 14.007, 15.999, 22.99, 30.974, 32.06, 35.45, 39.098};
const double kBiW1[] = {0.103, 0.105, 0.031, 0.749, 0.002, 0.002, 0.003, 0.003, 0.002};
const int kBiZ2[] = {1, 6, 7, 8, 11, 12, 15, 16, 20};
const double kBiA2[] = {1.008, 12.011, 14.007, 15.999, 22.99, 24.305, 30.974, 32.06, 40.078};
const double kBiW2[] = {0.03400000000000001, 0.15500000000000003, 0.04200000000000001,
                        0.43500000000000005, 0.0010000000000000002, 0.0020000000000000005,
                        0.10300000000000001, 0.0030000000000000005, 0.22500000000000003};
const omc_material kBuiltin[3] = {{2, kBiZ0, kBiA0, kBiW0, 75.0, 1.0},
                                  {9, kBiZ1, kBiA1, kBiW1, 75.3, 0.26},
                                  {9, kBiZ2, kBiA2, kBiW2, 110.0, 1.85}};
}  // namespace

int omc_create(omc_ctx** out, int nx, int ny, int nz, double dx, double dy, double dz,
               const float* density, const uint8_t* material, const omc_material* mats,
               int n_mats)
{
    if (!out) return fail(nullptr, OMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mats) {
        if (n_mats != 0 && n_mats != 3)
            return fail(nullptr, OMC_EINVAL, "mats == NULL selects the built-in library of 3 "
                                             "materials: pass n_mats 0 or 3");
        mats = kBuiltin;
        n_mats = 3;
    }
    if (nx < 1 || ny < 1 || nz < 1 || nx > OMC_MAX_DIM || ny > OMC_MAX_DIM || nz > OMC_MAX_DIM)
        return fail(nullptr, OMC_EINVAL, "phantom dimensions must be in 1..1024");
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz))
        return fail(nullptr, OMC_EINVAL, "voxel sizes must be finite and > 0");
    if (!density || !material) return fail(nullptr, OMC_EINVAL, "density/material is NULL");
    if (n_mats < 1 || n_mats > OMC_MAX_MATERIALS)
        return fail(nullptr, OMC_EINVAL, "need 1.." + std::to_string(OMC_MAX_MATERIALS) +
                                             " materials");
    omc_ctx* c = new (std::nothrow) omc_ctx();
    if (!c) return fail(nullptr, OMC_ENOMEM, "host allocation failed");
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->dx = dx;
    c->dy = dy;
    c->dz = dz;
    c->nvox = size_t(nx) * size_t(ny) * size_t(nz);
    c->mats.resize(n_mats);
    for (int m = 0; m < n_mats; ++m) {
        std::string why;
        if (validate_material(mats[m], c->mats[m], why) != OMC_OK) {
            delete c;
            return fail(nullptr, OMC_EINVAL, why);
        }
    }
    if (check_phantom(density, material, c->nvox, n_mats, c->rho_max)) {
        delete c;
        return fail(nullptr, OMC_EINVAL, "density must be finite and > 0 and material ids < n_mats");
    }
    omc_default_params(&c->prm);

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        delete c;
        return fail(nullptr, OMC_EDEVICE, "no HIP device available");
    }
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess) {
        delete c;
        return fail(nullptr, OMC_EDEVICE, "cannot query the HIP device");
    }
    // the fixed scratch of this device (omc_run_device_static); a failed
    // lookup leaves only that entry point unavailable
    c->d_scratch = scratch_of_device(c->device);
    bool ok = hipMalloc(&c->d_rho, c->nvox * sizeof(float)) == hipSuccess &&
              hipMalloc(&c->d_mat, c->nvox) == hipSuccess &&
              hipMalloc(&c->d_ctrl, 64 * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->d_counters, size_t(omc::kStatsRows) * omc::kNumCounters *
                                            sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc(&c->d_energies, size_t(omc::kStatsRows) * omc::kNumEnergies *
                                            sizeof(double)) == hipSuccess &&
              hipHostMalloc(&c->h_ctrl, 64 * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->d_run, sizeof(omc::RunDesc)) == hipSuccess &&
              hipMalloc(&c->d_order, 2 * omc::kSrcGroups * sizeof(uint32_t)) == hipSuccess &&
              hipHostMalloc(&c->h_run, sizeof(omc::RunDesc)) == hipSuccess;
    ok = ok && hipMalloc(&c->d_vox, c->nvox * 2 * sizeof(uint32_t)) == hipSuccess &&
         hipMalloc(&c->d_slot, omc::kMaxMaterials * sizeof(uint32_t)) == hipSuccess;
    ok = ok && upload_phantom(c, density, material) == OMC_OK;
    if (!ok) {
        omc_destroy(c);
        return fail(nullptr, OMC_ENOMEM, "device allocation or upload failed");
    }
    *out = c;
    return OMC_OK;
}

// Host densities and materials: finite and > 0, ids below n_mats; the
// largest density of each material (0 where it is absent).
int check_phantom(const float* density, const uint8_t* material, size_t nvox, int n_mats,
                  std::vector<double>& rmax)
{
    rmax.assign(n_mats, 0.0);
    for (size_t v = 0; v < nvox; ++v) {
        const float r = density[v];
        if (!(std::isfinite(r) && r > 0.0f) || material[v] >= n_mats) return OMC_EINVAL;
        rmax[material[v]] = std::max(rmax[material[v]], double(r));
    }
    return OMC_OK;
}

// The transport's voxel records from d_rho and d_mat: the tables hold the
// materials present (densities are > 0, so where the maximum is), in library
// order, and a voxel carries its material's slot. Synchronous, so that any
// stream may run next.
int build_vox(omc_ctx* c)
{
    c->present.clear();
    c->slot_of.assign(c->mats.size(), 0u);
    for (size_t m = 0; m < c->mats.size(); ++m)
        if (c->rho_max[m] > 0.0) {
            c->slot_of[m] = uint32_t(c->present.size());
            c->present.push_back(int(m));
        }
    uint32_t slot[omc::kMaxMaterials] = {};
    for (size_t m = 0; m < c->slot_of.size(); ++m) slot[m] = c->slot_of[m];
    HIP_TRY(c, hipMemcpy(c->d_slot, slot, sizeof slot, hipMemcpyHostToDevice));
    if (omc::launch_build_vox(c->d_rho, c->d_mat, c->nvox, c->d_slot, c->d_vox, nullptr))
        return fail(c, OMC_EDEVICE, "voxel record launch failed");
    HIP_TRY(c, hipStreamSynchronize(nullptr));
    // the majorant and the table slots depend on the phantom: new tables next run
    c->t32.valid = false;
    c->t64.valid = false;
    return OMC_OK;
}

// Host densities and materials to the device, then the voxel records.
int upload_phantom(omc_ctx* c, const float* density, const uint8_t* material)
{
    HIP_TRY(c, hipMemcpy(c->d_rho, density, c->nvox * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_mat, material, c->nvox, hipMemcpyHostToDevice));
    return build_vox(c);
}

int omc_set_phantom(omc_ctx* c, const float* density, const uint8_t* material)
{
    if (check_ctx(c) || !density || !material) return fail(c, OMC_EINVAL, "NULL argument");
    std::vector<double> rmax;
    if (check_phantom(density, material, c->nvox, int(c->mats.size()), rmax))
        return fail(c, OMC_EINVAL, "density must be finite and > 0 and material ids < n_mats");
    HIP_TRY(c, hipSetDevice(c->device));
    c->rho_max = rmax;
    return upload_phantom(c, density, material);
}

int omc_set_phantom_ct(omc_ctx* c, const int16_t* hu, int hu_on_device, const omc_ct_map* map)
{
    if (check_ctx(c) || !hu || !map) return fail(c, OMC_EINVAL, "NULL argument");
    const int nn = map->n_nodes, nb = map->n_bins;
    if (nn < 2 || nn > omc::kMaxCtNodes || !map->hu || !map->rho)
        return fail(c, OMC_EINVAL, "a CT map needs 2 <= n_nodes <= 64 calibration nodes");
    for (int k = 0; k < nn; ++k) {
        if (!std::isfinite(map->hu[k]) || (k > 0 && !(map->hu[k] > map->hu[k - 1])))
            return fail(c, OMC_EINVAL, "CT calibration HU values must be finite and increasing");
        if (!(map->rho[k] >= 1e-6 && map->rho[k] <= 100.0))
            return fail(c, OMC_EINVAL, "CT calibration densities must be in [1e-6, 100] g/cm3");
    }
    if (nb < 1 || nb > omc::kMaxCtBins || !map->material || (nb > 1 && !map->hu_upper))
        return fail(c, OMC_EINVAL, "a CT map needs 1 <= n_bins <= 32 material bins");
    for (int b = 0; b < nb; ++b) {
        if (map->material[b] < 0 || map->material[b] >= int(c->mats.size()))
            return fail(c, OMC_EINVAL, "CT bin material ids must be < n_mats");
        if (b + 1 < nb && (std::isnan(map->hu_upper[b]) ||
                           (b > 0 && !(map->hu_upper[b] > map->hu_upper[b - 1]))))
            return fail(c, OMC_EINVAL, "CT bin upper bounds must be increasing");
    }
    if (hu_on_device != 0 && hu_on_device != 1)
        return fail(c, OMC_EINVAL, "hu_on_device must be 0 or 1");
    HIP_TRY(c, hipSetDevice(c->device));
    if (hu_on_device && !device_range_ok(c, hu, c->nvox * sizeof(int16_t), alignof(int16_t)))
        return fail(c, OMC_EINVAL, "hu_on_device: the HU values must be an allocation of this "
                                   "context's device holding nx * ny * nz int16 values");
    // map [hu][rho][upper], bin materials, per-material maxima, and host HU
    // [hu][rho][upper][slopes]: the segment slopes are the definition's FP64
    // quotients, taken once here instead of per voxel
    std::vector<double> m(size_t(3 * nn - 1 + nb), 0.0);
    for (int k = 0; k < nn; ++k) {
        m[k] = map->hu[k];
        m[nn + k] = map->rho[k];
    }
    for (int b = 0; b + 1 < nb; ++b) m[2 * nn + b] = map->hu_upper[b];
    for (int k = 0; k + 1 < nn; ++k)
        m[2 * nn + nb + k] = (map->rho[k + 1] - map->rho[k]) / (map->hu[k + 1] - map->hu[k]);
    std::vector<uint32_t> bm(nb);
    for (int b = 0; b < nb; ++b) bm[b] = uint32_t(map->material[b]);
    const size_t o_mat = align256(m.size() * sizeof(double));
    const size_t o_max = o_mat + align256(bm.size() * sizeof(uint32_t));
    const size_t o_lr = o_max + align256(omc::kMaxMaterials * sizeof(uint32_t));
    const size_t o_lm = o_lr + align256(omc::kCtLutSize * sizeof(float));
    const size_t o_hu = o_lm + align256(omc::kCtLutSize * sizeof(uint8_t));
    const size_t total = o_hu + (hu_on_device ? 0 : c->nvox * sizeof(int16_t));
    char* buf = nullptr;
    if (hipMalloc(&buf, total) != hipSuccess) return fail(c, OMC_ENOMEM, "hipMalloc failed for the CT map");
    struct Guard {
        char* p;
        ~Guard() { dfree(p); }
    } guard{buf};
    const uint32_t zero[omc::kMaxMaterials] = {};
    HIP_TRY(c, hipMemcpy(buf, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(buf + o_mat, bm.data(), bm.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(buf + o_max, zero, sizeof zero, hipMemcpyHostToDevice));
    const int16_t* d_hu = hu;
    if (!hu_on_device) {
        HIP_TRY(c, hipMemcpy(buf + o_hu, hu, c->nvox * sizeof(int16_t), hipMemcpyHostToDevice));
        d_hu = reinterpret_cast<const int16_t*>(buf + o_hu);
    }
    if (omc::launch_ct_map(d_hu, c->nvox, reinterpret_cast<const double*>(buf),
                           reinterpret_cast<const uint32_t*>(buf + o_mat), nn, nb,
                           reinterpret_cast<float*>(buf + o_lr),
                           reinterpret_cast<uint8_t*>(buf + o_lm), c->d_rho, c->d_mat,
                           reinterpret_cast<uint32_t*>(buf + o_max), nullptr))
        return fail(c, OMC_EDEVICE, "CT mapping launch failed");
    uint32_t mx[omc::kMaxMaterials];
    HIP_TRY(c, hipMemcpy(mx, buf + o_max, sizeof mx, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < c->mats.size(); ++k) {
        float r;
        std::memcpy(&r, &mx[k], sizeof r);
        c->rho_max[k] = double(r);
    }
    return build_vox(c);
}

int omc_get_phantom(const omc_ctx* c, float* density, uint8_t* material)
{
    if (!c || !density || !material) return fail(nullptr, OMC_EINVAL, "NULL argument");
    if (hipSetDevice(c->device) != hipSuccess ||
        hipMemcpy(density, c->d_rho, c->nvox * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(material, c->d_mat, c->nvox, hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return fail(nullptr, OMC_EDEVICE, "cannot copy the phantom from the device");
    }
    return OMC_OK;
}

int omc_set_source(omc_ctx* c, const omc_source* s)
{
    if (check_ctx(c) || !s) return fail(c, OMC_EINVAL, "NULL argument");
    std::vector<double> edges, cdf;
    std::vector<float> psf;
    std::string why;
    if (check_source(s, edges, cdf, &psf, why) != OMC_OK) return fail(c, OMC_EINVAL, why);
    const bool dev = s->geometry == 2 && s->psf_on_device;
    if (dev) {
        HIP_TRY(c, hipSetDevice(c->device));
        const int rc = check_device_records(c, s->psf, s->n_psf, why);
        if (rc != OMC_OK) return fail(c, rc, why);
    }
    c->psf_dev = dev ? s->psf : nullptr;
    c->src = *s;
    c->src.edges = nullptr;
    c->src.weights = nullptr;
    c->src.psf = nullptr;
    c->edges = std::move(edges);
    c->cdf = std::move(cdf);
    c->psf = std::move(psf);
    c->psf_dirty = true;
    c->has_source = true;
    return OMC_OK;
}

int omc_set_params(omc_ctx* c, const omc_params* p)
{
    if (check_ctx(c) || !p) return fail(c, OMC_EINVAL, "NULL argument");
    if (!finite_pos(p->Eabs_e) || !finite_pos(p->Eabs_g) || !finite_pos(p->Wcc) ||
        !finite_pos(p->kc) || !finite_pos(p->dmax_s) || !(p->f_E > 0 && p->f_E < 1))
        return fail(c, OMC_EINVAL, "cut-offs and step limits must be positive, 0 < f_E < 1");
    if (p->Eabs_e < 2 * omc::kELo || p->Eabs_e > 10.0)
        return fail(c, OMC_EINVAL, "Eabs_e must be in [0.02, 10] MeV");
    if (p->n_batches < 1 || p->n_batches > OMC_MAX_BATCHES)
        return fail(c, OMC_EINVAL, "n_batches must be in 1..64");
    if (p->block_size < 64 || p->block_size > 256 || p->block_size % 64)
        return fail(c, OMC_EINVAL, "block_size must be 64, 128, 192 or 256");
    if (p->blocks_per_cu < 1 || p->blocks_per_cu > 32 || p->queue_factor < 1 ||
        p->queue_factor > 64 || p->chunk_histories < 0 || p->graph_depth < 0 ||
        p->graph_depth > 64 || p->beamlet_group < 0 || p->beamlet_group > 65535)
        return fail(c, OMC_EINVAL, "launch shape out of range");
    if (!(p->sparse_threshold >= 0.0 && p->sparse_threshold < 1.0))
        return fail(c, OMC_EINVAL, "sparse_threshold must be in [0, 1)");
    if (p->straggler_lanes < 0 || p->straggler_lanes > 63)
        return fail(c, OMC_EINVAL, "straggler_lanes must be in 0..63");
    if (p->electron_mode != 0 && p->electron_mode != 1)
        return fail(c, OMC_EINVAL, "electron_mode must be 0 or 1");
    if (p->table_mode < 0 || p->table_mode > 2)
        return fail(c, OMC_EINVAL, "table_mode must be 0, 1 or 2");
    if (p->photon_mode != 0 && p->photon_mode != 1)
        return fail(c, OMC_EINVAL, "photon_mode must be 0 or 1");
    if (p->tally_copies < 1 || p->tally_copies > 16 || (p->tally_copies & (p->tally_copies - 1)))
        return fail(c, OMC_EINVAL, "tally_copies must be 1, 2, 4, 8 or 16");
    if (p->source_order != 0 && p->source_order != 1)
        return fail(c, OMC_EINVAL, "source_order must be 0 or 1");
    if (p->event_lanes < 1 || p->event_lanes > 64)
        return fail(c, OMC_EINVAL, "event_lanes must be in 1..64");
    c->prm = *p;
    return OMC_OK;
}

int omc_get_geometry(const omc_ctx* c, int* nx, int* ny, int* nz, double* dx, double* dy,
                     double* dz)
{
    if (check_ctx(c)) return fail(nullptr, OMC_EINVAL, "NULL context");
    if (nx) *nx = c->nx;
    if (ny) *ny = c->ny;
    if (nz) *nz = c->nz;
    if (dx) *dx = c->dx;
    if (dy) *dy = c->dy;
    if (dz) *dz = c->dz;
    return OMC_OK;
}

int omc_get_params(const omc_ctx* c, omc_params* out)
{
    if (!c || !out) return fail(nullptr, OMC_EINVAL, "NULL argument");
    *out = c->prm;
    return OMC_OK;
}

int omc_run_device(omc_ctx* c, uint64_t n, uint32_t seed, uint32_t h0, double* d_dose,
                   double* d_dose2, void* hip_stream)
{
    if (check_ctx(c) || !d_dose || !d_dose2) return fail(c, OMC_EINVAL, "NULL argument");
    if (!c->has_source) return fail(c, OMC_ESTATE, "omc_set_source must be called first");
    if (n == 0 || uint64_t(h0) + n > (uint64_t(1) << 32))
        return fail(c, OMC_EINVAL, "need 1 <= n and h0 + n <= 2^32");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return c->prm.parity_fp64 ? run_impl<double>(c, n, seed, h0, d_dose, d_dose2, s)
                              : run_impl<float>(c, n, seed, h0, d_dose, d_dose2, s);
}

int omc_run_device_static(omc_ctx* c, uint64_t n, uint32_t seed, uint32_t h0, double* d_dose,
                          double* d_dose2, void* hip_stream)
{
    if (check_ctx(c) || !d_dose || !d_dose2) return fail(c, OMC_EINVAL, "NULL argument");
    if (!c->has_source) return fail(c, OMC_ESTATE, "omc_set_source must be called first");
    if (n == 0 || uint64_t(h0) + n > (uint64_t(1) << 32))
        return fail(c, OMC_EINVAL, "need 1 <= n and h0 + n <= 2^32");
    HIP_TRY(c, hipSetDevice(c->device));
    if (!c->d_scratch)
        return fail(c, OMC_EDEVICE, "the fixed device scratch is not available on this device");
    const size_t cells = size_t(c->prm.n_batches) * size_t(c->prm.tally_copies) * c->nvox;
    if (cells > kScrGridBytes / sizeof(double))
        return fail(c, OMC_EINVAL, "n_batches x tally_copies x voxels exceed the fixed scratch's "
                                   "tally region (6291456 doubles); use fewer batches or "
                                   "omc_run_device");
    if (!device_range_ok(c, d_dose, c->nvox * sizeof(double), sizeof(double)) ||
        !device_range_ok(c, d_dose2, c->nvox * sizeof(double), sizeof(double)))
        return fail(c, OMC_EINVAL, "dose and dose2 must each be nx*ny*nz doubles of device "
                                   "memory on the context's device");
    char* const b = c->d_scratch;
    RunMem M{};
    M.ctrl = reinterpret_cast<uint32_t*>(b + kScrCtrl);
    M.counters = reinterpret_cast<unsigned long long*>(b + kScrCounters);
    M.energies = reinterpret_cast<double*>(b + kScrEnergies);
    M.rows = kScratchRows;
    M.run = reinterpret_cast<omc::RunDesc*>(b + kScrRun);
    M.order = reinterpret_cast<uint32_t*>(b + kScrOrder);
    M.grid = reinterpret_cast<double*>(b + kScrGrid);
    M.fixed = true;
    M.src = b + kScrSrc;
    M.src_cap = kScrSrcBytes;
    M.queues = b + kScrQueues;
    M.queue_bytes = kScrQueueBytes;
    M.grid_cap = kScrGridBytes / sizeof(double);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return c->prm.parity_fp64 ? run_impl<double>(c, n, seed, h0, d_dose, d_dose2, s, &M)
                              : run_impl<float>(c, n, seed, h0, d_dose, d_dose2, s, &M);
}

int omc_run(omc_ctx* c, uint64_t n, uint32_t seed, uint32_t h0, double* dose, double* dose2)
{
    if (check_ctx(c) || !dose || !dose2) return fail(c, OMC_EINVAL, "NULL argument");
    HIP_TRY(c, hipSetDevice(c->device));
    if (!c->d_dose) {
        if (hipMalloc(&c->d_dose, c->nvox * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->d_dose2, c->nvox * sizeof(double)) != hipSuccess) {
            dfree(c->d_dose);
            dfree(c->d_dose2);
            return fail(c, OMC_ENOMEM, "hipMalloc failed for the dose grids");
        }
    }
    const int rc = omc_run_device(c, n, seed, h0, c->d_dose, c->d_dose2, nullptr);
    if (rc != OMC_OK && rc != OMC_ENUMERIC) return rc;
    HIP_TRY(c, hipMemcpy(dose, c->d_dose, c->nvox * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(dose2, c->d_dose2, c->nvox * sizeof(double), hipMemcpyDeviceToHost));
    return rc;
}

int omc_run_beamlets(omc_ctx* c, const omc_beamlet* b, int n_beamlets, uint32_t seed,
                     int on_device, void* hip_stream, omc_sparse_out* out)
{
    if (out) std::memset(out, 0, sizeof *out);
    if (check_ctx(c) || !b || !out) return fail(c, OMC_EINVAL, "NULL argument");
    if (n_beamlets < 1 || n_beamlets > 65535)
        return fail(c, OMC_EINVAL, "need 1 <= n_beamlets <= 65535");
    // validate every beamlet; spectra given by the same arrays are checked once
    std::vector<std::vector<double>> edges, cdf;
    std::vector<std::vector<float>> psfs;
    edges.reserve(n_beamlets);
    cdf.reserve(n_beamlets);
    psfs.reserve(n_beamlets + 1);
    psfs.emplace_back();  // the empty record list of analytic beamlets
    const float* last_r = nullptr;
    int last_nr = -1, last_dev = -1;
    std::vector<HostBeam> beams(n_beamlets);
    const double* last_e = nullptr;
    const double* last_w = nullptr;
    int last_n = -1;
    for (int i = 0; i < n_beamlets; ++i) {
        const omc_source& s = b[i].src;
        if (b[i].n_histories == 0 || uint64_t(b[i].h0) + b[i].n_histories > (uint64_t(1) << 32))
            return fail(c, OMC_EINVAL, "beamlet " + std::to_string(i) +
                                           ": need n_histories >= 1 and h0 + n <= 2^32");
        if (s.particle != b[0].src.particle)
            return fail(c, OMC_EINVAL, "all beamlets must have the same particle type");
        std::vector<double> e, w;
        std::vector<float> r;
        std::string why;
        // records given by the same array as the previous beamlet's are checked
        // and copied once (they share one device copy)
        const bool new_list = s.geometry == 2 && (s.psf != last_r || s.n_psf != last_nr ||
                                                  s.psf_on_device != last_dev);
        if (check_source(&s, e, w, new_list ? &r : nullptr, why) != OMC_OK)
            return fail(c, OMC_EINVAL, "beamlet " + std::to_string(i) + ": " + why);
        if (new_list) {
            if (s.psf_on_device) {
                HIP_TRY(c, hipSetDevice(c->device));
                const int rc = check_device_records(c, s.psf, s.n_psf, why);
                if (rc != OMC_OK) return fail(c, rc, "beamlet " + std::to_string(i) + ": " + why);
            }
            psfs.push_back(std::move(r));
            last_r = s.psf;
            last_nr = s.n_psf;
            last_dev = s.psf_on_device;
        }
        // beamlets that pass the same spectrum arrays share one device copy
        if (edges.empty() || s.n_bins == 0 || s.edges != last_e || s.weights != last_w ||
            s.n_bins != last_n) {
            edges.push_back(std::move(e));
            cdf.push_back(std::move(w));
            last_e = s.n_bins ? s.edges : nullptr;
            last_w = s.n_bins ? s.weights : nullptr;
            last_n = s.n_bins;
        }
        beams[i].src = s;
        beams[i].src.edges = nullptr;
        beams[i].src.weights = nullptr;
        beams[i].src.psf = nullptr;
        beams[i].psf = s.geometry == 2 ? &psfs.back() : &psfs.front();
        beams[i].psf_dev = s.geometry == 2 && s.psf_on_device ? s.psf : nullptr;
        beams[i].edges = &edges.back();
        beams[i].cdf = &cdf.back();
        beams[i].n = b[i].n_histories;
        beams[i].h0 = b[i].h0;
    }
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return c->prm.parity_fp64
               ? beamlets_impl<double>(c, beams, b[0].src.particle, seed, on_device != 0, s, out)
               : beamlets_impl<float>(c, beams, b[0].src.particle, seed, on_device != 0, s, out);
}

void omc_free_sparse(omc_sparse_out* out)
{
    if (!out) return;
    std::free(out->row_ptr);
    if (out->on_device) {
        if (out->voxel) (void)hipFree(out->voxel);
        if (out->dose) (void)hipFree(out->dose);
    } else {
        std::free(out->voxel);
        std::free(out->dose);
    }
    std::memset(out, 0, sizeof *out);
}

int omc_autotune(omc_ctx* c, uint64_t n_probe, uint32_t seed, omc_params* best)
{
    if (check_ctx(c)) return fail(c, OMC_EINVAL, "NULL context");
    if (!c->has_source) return fail(c, OMC_ESTATE, "omc_set_source must be called first");
    if (n_probe == 0 || n_probe > (uint64_t(1) << 31))
        return fail(c, OMC_EINVAL, "need 1 <= n_probe <= 2^31");
    HIP_TRY(c, hipSetDevice(c->device));
    if (!c->d_dose) {
        if (hipMalloc(&c->d_dose, c->nvox * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->d_dose2, c->nvox * sizeof(double)) != hipSuccess) {
            dfree(c->d_dose);
            dfree(c->d_dose2);
            return fail(c, OMC_ENOMEM, "hipMalloc failed for the dose grids");
        }
    }
    const omc_params base = c->prm;
    // generations a chunk needs when driven to empty queues from the host
    auto timed = [&](const omc_params& p, double& ms, omc_counters& L) {
        c->prm = p;
        double bestms = 1e300;
        for (int r = 0; r < 3; ++r) {  // the first run builds tables, queues and graph
            const auto t0 = std::chrono::steady_clock::now();
            const int rc = omc_run_device(c, n_probe, seed, 0, c->d_dose, c->d_dose2, nullptr);
            const auto t1 = std::chrono::steady_clock::now();
            if (rc != OMC_OK) return rc;
            if (r > 0) bestms = std::min(bestms, std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        ms = bestms;
        L = c->last;
        return int(OMC_OK);
    };
    struct Shape {
        int block, per_cu;
    };
    const Shape shapes[] = {{256, 2}, {256, 4}, {256, 6}, {256, 8}, {128, 4}, {128, 8}};
    // the largest chunk tried: the whole probe while its queues (four of them,
    // at the probing queue factor of 8) take at most half the free device
    // memory; fewer, longer persistent launches leave fewer tails of
    // long-lived particles
    uint64_t full = std::min<uint64_t>(n_probe, uint64_t(1) << 24);
    {
        size_t free_b = 0, total_b = 0;
        (void)hipMemGetInfo(&free_b, &total_b);
        (void)hipGetLastError();
        const size_t per = c->prm.parity_fp64 ? 8 * sizeof(double) + 6 * sizeof(uint32_t)
                                              : 8 * sizeof(float) + 6 * sizeof(uint32_t);
        const uint64_t fit = uint64_t(free_b / 2 / (4 * 8 * per));
        full = std::max(full, std::min<uint64_t>(n_probe, std::min<uint64_t>(fit, 0x0fffffffull)));
    }
    omc_params top = base;
    double top_ms = 1e300;
    uint64_t hwm = 0, hwm_chunk = 1;
    int last_rc = OMC_OK;
    for (const Shape& sh : shapes) {
        omc_params p = base;
        p.block_size = sh.block;
        p.blocks_per_cu = sh.per_cu;
        p.queue_factor = std::max(base.queue_factor, 8);
        p.timing = 0;
        // host-driven generations first: they also give the generations per chunk
        p.graph_depth = 0;
        p.chunk_histories = int(full);
        double ms;
        omc_counters L;
        int rc = timed(p, ms, L);
        if (rc != OMC_OK) {
            last_rc = rc;
            continue;
        }
        const uint64_t chunks = (n_probe + full - 1) / full;
        const int per_chunk = int(std::min<uint64_t>(64, (L.iterations + chunks - 1) / chunks));
        std::vector<omc_params> cand;
        cand.push_back(p);
        const uint64_t divs[] = {1, 2, 4, 8};
        for (uint64_t d : divs) {
            const uint64_t S = std::max<uint64_t>(1, full / d);
            const int ks[] = {per_chunk, std::max(1, per_chunk / 2), 3, 2};
            for (int k : ks) {
                omc_params q = p;
                q.chunk_histories = int(S);
                q.graph_depth = std::max(1, std::min(64, k));
                bool dup = false;
                for (const auto& o : cand)
                    dup = dup || (o.chunk_histories == q.chunk_histories &&
                                  o.graph_depth == q.graph_depth);
                if (!dup) cand.push_back(q);
            }
        }
        for (size_t i = 0; i < cand.size(); ++i) {
            if (i > 0) {
                rc = timed(cand[i], ms, L);
                if (rc != OMC_OK) {
                    last_rc = rc;
                    continue;
                }
            }
            const uint64_t S = uint64_t(cand[i].chunk_histories);
            if (double(L.queue_hwm_ph + L.queue_hwm_el) / double(S) >
                double(hwm) / double(hwm_chunk)) {
                hwm = L.queue_hwm_ph + L.queue_hwm_el;
                hwm_chunk = S;
            }
            if (ms < top_ms) {
                top_ms = ms;
                top = cand[i];
            }
        }
    }
    // private tally copies: they pay where the deposits crowd a few voxels (a
    // narrow beam); tried on the fastest shape while the grids take at most a
    // quarter of the free device memory
    if (top_ms < 1e300) {
        size_t free_b = 0, total_b = 0;
        (void)hipMemGetInfo(&free_b, &total_b);
        (void)hipGetLastError();
        for (int k : {2, 4, 8}) {
            const size_t bytes = size_t(base.n_batches) * size_t(k) * c->nvox * sizeof(double);
            if (bytes > free_b / 4) break;
            omc_params q = top;
            q.tally_copies = k;
            double ms;
            omc_counters L;
            if (timed(q, ms, L) != OMC_OK) continue;
            if (ms < top_ms) {
                top_ms = ms;
                top = q;
            }
        }
        // the number of waiting electrons that starts an event pass
        for (int k : {8, 24, 32}) {
            omc_params q = top;
            q.event_lanes = k;
            double ms;
            omc_counters L;
            if (timed(q, ms, L) == OMC_OK && ms < top_ms) {
                top_ms = ms;
                top = q;
            }
        }
        // the other source order, where the source energies differ
        if (c->src.geometry == 2 || c->src.n_bins > 0) {
            omc_params q = top;
            q.source_order = 1 - top.source_order;
            double ms;
            omc_counters L;
            if (timed(q, ms, L) == OMC_OK && ms < top_ms) {
                top_ms = ms;
                top = q;
            }
        }
    }
    drop_graph(c);
    if (top_ms >= 1e300) {
        c->prm = base;
        return last_rc != OMC_OK ? last_rc : fail(c, OMC_EDEVICE, "no candidate completed");
    }
    // queue capacity: the largest occupancy per chunk history seen, with margin
    const double per_hist = double(hwm) / double(hwm_chunk);
    top.queue_factor = int(std::min(64.0, std::max(2.0, std::ceil(1.5 * per_hist + 1.0))));
    top.timing = base.timing;
    c->prm = top;
    if (best) *best = top;
    return OMC_OK;
}

int omc_get_counters(const omc_ctx* c, omc_counters* out)
{
    if (!c || !out) return fail(nullptr, OMC_EINVAL, "NULL argument");
    *out = c->last;
    return OMC_OK;
}

int omc_get_timing(const omc_ctx* c, omc_timing* out)
{
    if (!c || !out) return fail(nullptr, OMC_EINVAL, "NULL argument");
    *out = c->timing;
    return OMC_OK;
}

int omc_debug_philox(uint32_t seed, uint32_t h, uint64_t q, uint32_t n0, uint32_t nblocks,
                     uint32_t* out)
{
    if (!out || nblocks == 0 || nblocks > (1u << 24))
        return fail(nullptr, OMC_EINVAL, "need out != NULL and 1 <= nblocks <= 2^24");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(nullptr, OMC_EDEVICE, "no HIP device available");
    uint32_t* d = nullptr;
    if (hipMalloc(&d, size_t(nblocks) * 4 * sizeof(uint32_t)) != hipSuccess)
        return fail(nullptr, OMC_ENOMEM, "hipMalloc failed");
    int rc = OMC_OK;
    if (omc::launch_philox_debug(seed, h, q, n0, nblocks, d, nullptr) ||
        hipMemcpy(out, d, size_t(nblocks) * 4 * sizeof(uint32_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
        rc = fail(nullptr, OMC_EDEVICE, "Philox debug kernel failed");
    (void)hipFree(d);
    return rc;
}

int omc_debug_sample(omc_ctx* c, int which, const double* args, uint32_t seed, uint32_t n,
                     double* out, uint32_t* words)
{
    if (check_ctx(c) || !out || !words || n == 0 || n > (1u << 22))
        return fail(c, OMC_EINVAL, "need a context, out and words, and 1 <= n <= 2^22");
    if (which < omc::SMP_COMPTON || which > omc::SMP_SOURCE)
        return fail(c, OMC_EINVAL, "unknown sampler");
    if (which == omc::SMP_SOURCE) {
        if (!c->has_source) return fail(c, OMC_ESTATE, "omc_set_source must be called first");
    } else {
        if (!args) return fail(c, OMC_EINVAL, "NULL args");
        const double nrm = std::sqrt(args[1] * args[1] + args[2] * args[2] + args[3] * args[3]);
        if (!(args[0] > 0.0 && args[0] <= omc::kEHi) || !(std::fabs(nrm - 1.0) < 1e-6))
            return fail(c, OMC_EINVAL, "need 0 < E <= 20 MeV and a unit direction");
        if (which == omc::SMP_PAIR && !(args[0] > 2.0 * omc::kMC2))
            return fail(c, OMC_EINVAL, "pair production needs E > 2 mc^2");
        if (which == omc::SMP_MS && !(args[4] > 0.0 && std::isfinite(args[4])))
            return fail(c, OMC_EINVAL, "multiple scattering needs x = s / lambda_1 > 0");
    }
    HIP_TRY(c, hipSetDevice(c->device));
    std::memset(out, 0, size_t(n) * omc::kSampleWords * sizeof(double));
    return c->prm.parity_fp64 ? debug_sample_impl<double>(c, which, args, seed, n, out, words)
                              : debug_sample_impl<float>(c, which, args, seed, n, out, words);
}

int omc_debug_trace(omc_ctx* c, uint32_t seed, uint32_t h, double* out, uint32_t max_records,
                    uint32_t* n_records)
{
    if (check_ctx(c) || !out || !n_records || max_records == 0 || max_records > (1u << 24))
        return fail(c, OMC_EINVAL, "invalid trace arguments");
    if (!c->has_source) return fail(c, OMC_ESTATE, "omc_set_source must be called first");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t bytes = size_t(max_records) * omc::kTraceWords * sizeof(double);
    double* d_buf = nullptr;
    uint32_t* d_n = nullptr;
    double *d_dose = nullptr, *d_dose2 = nullptr;
    int rc = OMC_OK;
    if (hipMalloc(&d_buf, bytes) != hipSuccess || hipMalloc(&d_n, sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&d_dose, c->nvox * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_dose2, c->nvox * sizeof(double)) != hipSuccess) {
        rc = fail(c, OMC_ENOMEM, "hipMalloc failed for the trace");
    } else if (hipMemset(d_n, 0, sizeof(uint32_t)) != hipSuccess) {
        rc = fail(c, OMC_EDEVICE, "hipMemset failed");
    } else {
        c->trace = omc::TraceView{d_buf, d_n, max_records, h, 1};
        rc = c->prm.parity_fp64 ? run_impl<double>(c, 1, seed, h, d_dose, d_dose2, nullptr)
                                : run_impl<float>(c, 1, seed, h, d_dose, d_dose2, nullptr);
        c->trace = omc::TraceView{};
        uint32_t n = 0;
        if (rc == OMC_OK &&
            (hipMemcpy(&n, d_n, sizeof n, hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(out, d_buf, size_t(std::min(n, max_records)) * omc::kTraceWords *
                                       sizeof(double), hipMemcpyDeviceToHost) != hipSuccess))
            rc = fail(c, OMC_EDEVICE, "trace readback failed");
        *n_records = std::min(n, max_records);
    }
    dfree(d_buf);
    dfree(d_n);
    dfree(d_dose);
    dfree(d_dose2);
    return rc;
}

int omc_host_tables(const omc_material* mat, double Wcc, double kc, double* out)
{
    if (!mat || !out || !finite_pos(Wcc) || !finite_pos(kc))
        return fail(nullptr, OMC_EINVAL, "invalid argument");
    omc::MaterialSpec m;
    std::string why;
    if (validate_material(*mat, m, why) != OMC_OK) return fail(nullptr, OMC_EINVAL, why);
    const omc::MaterialTables t = omc::build_material_tables(m, Wcc, kc);
    const std::array<double, omc::kNE>* rows[OMC_TABLE_ROWS] = {
        &t.muC, &t.muPE, &t.muPair, &t.muTot, &t.Scol, &t.Srad, &t.R, &t.sigM, &t.sigB, &t.sigHat,
        &t.K1};
    for (int r = 0; r < OMC_TABLE_ROWS; ++r)
        std::memcpy(out + size_t(r) * omc::kNE, rows[r]->data(), omc::kNE * sizeof(double));
    return OMC_OK;
}

int omc_host_ms_table(double* out)
{
    if (!out) return fail(nullptr, OMC_EINVAL, "out is NULL");
    const auto t = omc::build_ms_table();
    std::memcpy(out, t.data(), t.size() * sizeof(double));
    return OMC_OK;
}

const char* omc_last_error(const omc_ctx* c)
{
    if (c) return c->err.c_str();
    return g_thread_error.c_str();
}

void omc_destroy(omc_ctx* c)
{
    if (!c) return;
    free_tables(c->t32);
    free_tables(c->t64);
    free_queues(c->q32);
    free_queues(c->q64);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    dfree(c->d_rho);
    dfree(c->d_mat);
    dfree(c->d_vox);
    dfree(c->d_slot);
    dfree(c->d_src);
    dfree(c->d_psf);
    dfree(c->d_chk);
    dfree(c->d_run);
    dfree(c->d_cscratch);
    dfree(c->d_grid);
    dfree(c->d_dose);
    dfree(c->d_dose2);
    dfree(c->d_ctrl);
    dfree(c->d_order);
    dfree(c->d_counters);
    dfree(c->d_energies);
    if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
    if (c->h_run) (void)hipHostFree(c->h_run);
    delete c;
}

}  // extern "C"
