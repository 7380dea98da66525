// runtime.cpp -- host runtime and C ABI (include/omc.h) of the gfx950 engine.
//
// One context per phantom. A run (Table 1 of the paper, re-shaped):
//   for each chunk of source histories:
//     source kernel -> photon or electron queue
//     repeat: photon kernel (photon queue -> electrons, annihilation photons)
//             electron kernel (electron queue -> deltas, bremsstrahlung and
//             annihilation photons); swap queues; read the queue counts
//     until both queues are empty
//   fold the FP64 batch grids into dose and dose^2.
// The paper picks the largest of {photon stack, electron stack, source} per
// iteration and launches M same-type work-items; here each generation drains a
// whole queue with a persistent grid that keeps every lane busy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
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
    R* K1 = nullptr;
    R* msA = nullptr;
    R* Rabs = nullptr;
    R* edges = nullptr;
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
    std::vector<float> rho;
    std::vector<uint8_t> mat;
    std::vector<omc::MaterialSpec> mats;
    std::vector<double> rho_max;  // per material

    bool has_source = false;
    omc_source src{};
    std::vector<double> edges, weights, cdf;
    omc_params prm{};

    int cu_count = 0;
    float* d_rho = nullptr;
    uint8_t* d_mat = nullptr;
    double* d_cdf = nullptr;
    double* d_grid = nullptr;
    size_t grid_batches = 0;
    double* d_dose = nullptr;   // fold target of omc_run
    double* d_dose2 = nullptr;
    uint32_t* d_ctrl = nullptr;  // [4][count, head], overflow at [8]
    unsigned long long* d_counters = nullptr;
    double* d_energies = nullptr;
    uint32_t* h_ctrl = nullptr;  // pinned readback

    // host-side tables (FP64) for the current Wcc, kc, Eabs_e
    std::vector<omc::MaterialTables> tabs;
    std::array<double, omc::kNA> ms{};
    double tab_Wcc = -1, tab_kc = -1, tab_Eabs = -1;
    std::vector<double> Rabs;

    DeviceTables<float> t32;
    DeviceTables<double> t64;
    DeviceQueues<float> q32;
    DeviceQueues<double> q64;

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
    dfree(t.K1);
    dfree(t.msA);
    dfree(t.Rabs);
    dfree(t.edges);
    t.valid = false;
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

template <typename R>
int device_tables(omc_ctx* c, DeviceTables<R>& t)
{
    host_tables(c);
    if (t.valid) return OMC_OK;
    const int nm = int(c->mats.size());
    const int NE = omc::kNE;
    std::vector<R> ph(size_t(nm) * NE * 4), el(size_t(nm) * NE * 4), K1(size_t(nm) * NE),
        muhat(NE), msA(omc::kNA), Rabs(nm);
    for (int m = 0; m < nm; ++m) {
        const auto& T = c->tabs[m];
        for (int i = 0; i < NE; ++i) {
            const size_t o = (size_t(m) * NE + i) * 4;
            ph[o + 0] = R(T.muTot[i]);
            ph[o + 1] = R(T.muC[i]);
            ph[o + 2] = R(T.muPE[i]);
            ph[o + 3] = R(0);
            el[o + 0] = R(T.R[i]);
            el[o + 1] = R(T.sigHat[i]);
            el[o + 2] = R(T.sigM[i]);
            el[o + 3] = R(T.sigB[i]);
            K1[size_t(m) * NE + i] = R(T.K1[i]);
        }
        Rabs[m] = R(c->Rabs[m]);
    }
    // photon majorant over the materials present: node-wise max of
    // rho_max(m) * mu_tot(m), whose interpolant bounds every material's
    for (int i = 0; i < NE; ++i) {
        double mx = 0.0;
        for (int m = 0; m < nm; ++m) mx = std::max(mx, c->rho_max[m] * c->tabs[m].muTot[i]);
        muhat[i] = R(mx);
    }
    for (int j = 0; j < omc::kNA; ++j) msA[j] = R(c->ms[j]);
    int rc;
    if ((rc = upload(c, t.ph, ph)) || (rc = upload(c, t.el, el)) || (rc = upload(c, t.K1, K1)) ||
        (rc = upload(c, t.muhat, muhat)) || (rc = upload(c, t.msA, msA)) ||
        (rc = upload(c, t.Rabs, Rabs)))
        return rc;
    t.valid = true;
    return OMC_OK;
}

template <typename R>
int ensure_queues(omc_ctx* c, DeviceQueues<R>& Q, uint32_t cap_ph, uint32_t cap_el)
{
    if (Q.mem && Q.cap_ph >= cap_ph && Q.cap_el >= cap_el) return OMC_OK;
    free_queues(Q);
    const size_t per = 7 * sizeof(R) + 4 * sizeof(uint32_t) + 1;
    const size_t bytes = (size_t(cap_ph) * 2 + size_t(cap_el) * 2) * per + 64 * 16;
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
        q.type = reinterpret_cast<uint8_t*>(take(cap));
        q.cap = cap;
        q.count = c->d_ctrl + 2 * k;
        q.head = c->d_ctrl + 2 * k + 1;
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

struct EventTimer {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
    hipEvent_t first = nullptr, last = nullptr;
    void begin(int kind)
    {
        if (!on) return;
        hipEvent_t a, b;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, s);
        ev.push_back({kind, {a, b}});
        if (!first) first = a;
    }
    void end()
    {
        if (!on) return;
        (void)hipEventRecord(ev.back().second.second, s);
        last = ev.back().second.second;
    }
    void collect(omc_timing& t)
    {
        t = omc_timing{};
        if (!on) return;
        for (auto& e : ev) {
            float ms = 0;
            (void)hipEventSynchronize(e.second.second);
            (void)hipEventElapsedTime(&ms, e.second.first, e.second.second);
            t.launches[e.first] += 1;
            t.total_ms[e.first] += ms;
        }
        if (first && last) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, first, last);
            t.run_ms = ms;
        }
        for (auto& e : ev) {
            (void)hipEventDestroy(e.second.first);
            (void)hipEventDestroy(e.second.second);
        }
        ev.clear();
    }
};

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
    &omc_counters::push_el,     &omc_counters::src_miss,      &omc_counters::watchdog};

template <typename R>
int run_impl(omc_ctx* c, uint64_t N, uint32_t seed, uint32_t h0, double* d_dose, double* d_dose2,
             hipStream_t s)
{
    DeviceTables<R>& T = tables_of(c, R());
    DeviceQueues<R>& Q = queues_of(c, R());
    int rc = device_tables(c, T);
    if (rc) return rc;
    const omc_params& P = c->prm;
    const int B = P.n_batches;
    const uint64_t chunk =
        P.chunk_histories > 0 ? uint64_t(P.chunk_histories) : std::min<uint64_t>(N, uint64_t(1) << 24);
    const uint64_t S = std::min<uint64_t>(chunk, N);
    // capacity: secondaries per source history, plus the holes left by the
    // per-wave slot reservations of the two kernels that append to a queue
    const uint64_t waves = uint64_t(c->cu_count) * P.blocks_per_cu * (P.block_size / 64);
    const uint64_t qcap = std::min<uint64_t>(
        uint64_t(P.queue_factor) * S + 2 * waves * omc::kResBlockSlots + 4096, 0x7fffffffull);
    if ((rc = ensure_queues(c, Q, uint32_t(std::max<uint64_t>(qcap, S)), uint32_t(qcap)))) return rc;

    // tally grids
    const size_t need = size_t(B) * c->nvox;
    if (c->grid_batches < size_t(B)) {
        dfree(c->d_grid);
        if (hipMalloc(&c->d_grid, need * sizeof(double)) != hipSuccess) {
            c->d_grid = nullptr;
            c->grid_batches = 0;
            return fail(c, OMC_ENOMEM, "hipMalloc failed for the batch dose grids");
        }
        c->grid_batches = size_t(B);
    }
    // source spectrum edges in the transport precision
    if (c->src.n_bins > 0 && !T.edges) {
        std::vector<R> e(c->edges.begin(), c->edges.end());
        if ((rc = upload(c, T.edges, e))) return rc;
    }

    EventTimer tm;
    tm.on = P.timing != 0;
    tm.s = s;

    HIP_TRY(c, hipMemsetAsync(c->d_grid, 0, need * sizeof(double), s));
    HIP_TRY(c, hipMemsetAsync(c->d_counters, 0,
                              size_t(omc::kStatsRows) * omc::kNumCounters *
                                  sizeof(unsigned long long), s));
    HIP_TRY(c, hipMemsetAsync(c->d_energies, 0,
                              size_t(omc::kStatsRows) * omc::kNumEnergies * sizeof(double), s));
    HIP_TRY(c, hipMemsetAsync(c->d_ctrl, 0, 16 * sizeof(uint32_t), s));

    omc::KernelArgs<R> a{};
    a.ph = {c->d_rho, c->d_mat, c->nx, c->ny, c->nz, R(c->dx), R(c->dy), R(c->dz),
            R(1.0 / c->dx), R(1.0 / c->dy), R(1.0 / c->dz)};
    const omc::EnergyGrid g = omc::energy_grid();
    a.tab.ph = T.ph;
    a.tab.muhat = T.muhat;
    a.tab.el = T.el;
    a.tab.K1 = T.K1;
    a.tab.msA = T.msA;
    a.tab.Rabs = T.Rabs;
    a.tab.n_mats = int(c->mats.size());
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
    a.tally = {c->d_grid, c->nvox, N, h0, B};
    a.stats = {c->d_counters, c->d_energies, omc::kStatsRows, c->d_ctrl + 8, c->d_ctrl + 9};
    const omc_source& sr = c->src;
    a.src.cdf = c->d_cdf;
    a.src.edges = T.edges;
    a.src.n_bins = sr.n_bins;
    a.src.particle = sr.particle;
    a.src.point = sr.geometry == 1;
    a.src.mono_E = R(sr.mono_E);
    a.src.ssd = R(sr.ssd);
    a.src.z_field = R(sr.z_field);
    a.src.fx = R(sr.fx);
    a.src.fy = R(sr.fy);
    a.src.cx = R(sr.cx);
    a.src.cy = R(sr.cy);
    a.src.sx = R(sr.sx);
    a.src.sy = R(sr.sy);
    a.src.rotate = sr.gantry_deg != 0.0;
    const double gr = sr.gantry_deg * omc::kPi / 180.0;
    a.src.cg = R(std::cos(gr));
    a.src.sg = R(std::sin(gr));
    a.src.iso_x = R(sr.iso_x);
    a.src.iso_z = R(sr.iso_z);
    a.trace = c->trace;
    a.seed = seed;
    a.chunk = 64;

    const int block = P.block_size;
    const int tgrid = c->cu_count * P.blocks_per_cu;
    // a generation with few records needs fewer persistent work-groups: about
    // two records per lane, never fewer than one work-group per CU
    auto grid_for = [&](uint32_t n_records) {
        const uint64_t want = (uint64_t(n_records) + 2ull * block - 1) / (2ull * block);
        return int(std::max<uint64_t>(c->cu_count, std::min<uint64_t>(want, uint64_t(tgrid))));
    };
    const int nm = int(c->mats.size());
    const size_t lds_ph = omc::photon_lds_bytes<R>(nm);
    const size_t lds_el = omc::electron_lds_bytes<R>(nm);
    int lds_max = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    if (lds_ph > size_t(lds_max) || lds_el > size_t(lds_max))
        return fail(c, OMC_EUNSUP, "material tables exceed the LDS of a work-group; use fewer "
                                   "materials (or the FP32 build)");

    omc_counters& L = c->last;
    L = omc_counters{};
    uint32_t iters = 0;
    for (uint64_t done = 0; done < N; done += S) {
        const uint32_t cnt = uint32_t(std::min<uint64_t>(S, N - done));
        int pc = 0, ec = 2;  // current photon / electron buffers
        a.qp_out = Q.q[pc];
        a.qe_out = Q.q[ec];
        a.src_begin = uint32_t(done);
        a.src_count = cnt;
        tm.begin(0);
        if (omc::Launch<R>::source(a, int((cnt + 255) / 256), 256, s))
            return fail(c, OMC_EDEVICE, "source kernel launch failed");
        tm.end();
        uint32_t n_ph = sr.particle == 0 ? cnt : 0, n_el = sr.particle == 0 ? 0 : cnt;
        for (;;) {
            if (++iters > 100000) return fail(c, OMC_ENUMERIC, "generation limit exceeded");
            if (n_ph) {
                a.qin = Q.q[pc];
                a.qe_out = Q.q[ec];
                a.qp_out = Q.q[pc ^ 1];
                tm.begin(1);
                if (omc::Launch<R>::photon(a, grid_for(n_ph), block, lds_ph, s))
                    return fail(c, OMC_EDEVICE, "photon kernel launch failed");
                tm.end();
            }
            // electrons created by the photon kernel are in Q.q[ec]; their count
            // is known on the host only when no photon kernel ran before
            a.qin = Q.q[ec];
            a.qe_out = Q.q[ec ^ 1];
            a.qp_out = Q.q[pc ^ 1];
            tm.begin(2);
            if (omc::Launch<R>::electron(a, n_ph ? tgrid : grid_for(n_el), block, lds_el, s))
                return fail(c, OMC_EDEVICE, "electron kernel launch failed");
            tm.end();
            if (omc::launch_queue_reset(c->d_ctrl, (1 << pc) | (1 << ec), s))
                return fail(c, OMC_EDEVICE, "queue reset launch failed");
            pc ^= 1;
            ec ^= 1;
            HIP_TRY(c, hipMemcpyAsync(c->h_ctrl, c->d_ctrl, 16 * sizeof(uint32_t),
                                      hipMemcpyDeviceToHost, s));
            HIP_TRY(c, hipStreamSynchronize(s));
            if (c->h_ctrl[8]) {
                tm.collect(c->timing);
                return fail(c, OMC_EQUEUE,
                            "secondary particle queue overflow; raise queue_factor or lower "
                            "chunk_histories");
            }
            n_ph = c->h_ctrl[2 * pc];
            n_el = c->h_ctrl[2 * ec];
            L.queue_hwm_ph = std::max<uint64_t>(L.queue_hwm_ph, n_ph);
            L.queue_hwm_el = std::max<uint64_t>(L.queue_hwm_el, n_el);
            if (n_ph == 0 && n_el == 0) break;
        }
    }
    std::vector<double> nb;
    batch_sizes(N, B, nb);
    tm.begin(3);
    if (omc::launch_fold(c->d_grid, c->d_rho, c->nvox, B, nb.data(), c->dx * c->dy * c->dz,
                         double(N), d_dose, d_dose2, s))
        return fail(c, OMC_EDEVICE, "fold kernel launch failed");
    tm.end();
    unsigned long long cnts[omc::kNumCounters];
    double en[omc::kNumEnergies];
    if (omc::launch_stats_reduce(c->d_counters, c->d_energies, omc::kStatsRows, s))
        return fail(c, OMC_EDEVICE, "statistics reduce launch failed");
    HIP_TRY(c, hipMemcpyAsync(c->h_ctrl, c->d_ctrl, 16 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                              s));
    HIP_TRY(c, hipMemcpyAsync(cnts, c->d_counters, sizeof cnts, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(en, c->d_energies, sizeof en, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    tm.collect(c->timing);
    for (int k = 0; k < omc::kNumCounters; ++k) L.*kCounterField[k] = cnts[k];
    L.E_incident = en[omc::EN_INCIDENT];
    L.E_deposited = en[omc::EN_DEPOSITED];
    L.E_escaped = en[omc::EN_ESCAPED];
    L.E_pair_rest = double(L.ph_pair) * 2.0 * omc::kMC2;
    L.E_annih_rest = double(L.pos_annihil) * 2.0 * omc::kMC2;
    L.iterations = iters;
    L.max_steps = c->h_ctrl[9];
    const double lhs = L.E_incident + L.E_annih_rest - L.E_pair_rest;
    const double rhs = L.E_deposited + L.E_escaped;
    if (!std::isfinite(lhs) || !std::isfinite(rhs) || std::fabs(lhs - rhs) > 1e-9 * std::fabs(lhs))
        return fail(c, OMC_ENUMERIC, "energy ledger violated: incident+annihilation-pair != "
                                     "deposited+escaped");
    return OMC_OK;
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
}

int omc_create(omc_ctx** out, int nx, int ny, int nz, double dx, double dy, double dz,
               const float* density, const uint8_t* material, const omc_material* mats,
               int n_mats)
{
    if (!out) return fail(nullptr, OMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1 || nx > OMC_MAX_DIM || ny > OMC_MAX_DIM || nz > OMC_MAX_DIM)
        return fail(nullptr, OMC_EINVAL, "phantom dimensions must be in 1..1024");
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz))
        return fail(nullptr, OMC_EINVAL, "voxel sizes must be finite and > 0");
    if (!density || !material) return fail(nullptr, OMC_EINVAL, "density/material is NULL");
    if (n_mats < 1 || n_mats > OMC_MAX_MATERIALS || !mats)
        return fail(nullptr, OMC_EINVAL, "need 1..8 materials");
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
    c->rho.assign(density, density + c->nvox);
    c->mat.assign(material, material + c->nvox);
    c->rho_max.assign(n_mats, 0.0);
    for (size_t v = 0; v < c->nvox; ++v) {
        const float r = c->rho[v];
        if (!(std::isfinite(r) && r > 0.0f) || c->mat[v] >= n_mats) {
            delete c;
            return fail(nullptr, OMC_EINVAL,
                        "density must be finite and > 0 and material ids < n_mats");
        }
        c->rho_max[c->mat[v]] = std::max(c->rho_max[c->mat[v]], double(r));
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
    bool ok = hipMalloc(&c->d_rho, c->nvox * sizeof(float)) == hipSuccess &&
              hipMalloc(&c->d_mat, c->nvox) == hipSuccess &&
              hipMalloc(&c->d_ctrl, 64 * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->d_counters, size_t(omc::kStatsRows) * omc::kNumCounters *
                                            sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc(&c->d_energies, size_t(omc::kStatsRows) * omc::kNumEnergies *
                                            sizeof(double)) == hipSuccess &&
              hipHostMalloc(&c->h_ctrl, 64 * sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMemcpy(c->d_rho, c->rho.data(), c->nvox * sizeof(float), hipMemcpyHostToDevice) ==
                   hipSuccess;
    ok = ok && hipMemcpy(c->d_mat, c->mat.data(), c->nvox, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        omc_destroy(c);
        return fail(nullptr, OMC_ENOMEM, "device allocation or upload failed");
    }
    *out = c;
    return OMC_OK;
}

int omc_set_source(omc_ctx* c, const omc_source* s)
{
    if (check_ctx(c) || !s) return fail(c, OMC_EINVAL, "NULL argument");
    if (s->particle != 0 && s->particle != 1) return fail(c, OMC_EINVAL, "particle must be 0 or 1");
    if (s->geometry != 0 && s->geometry != 1) return fail(c, OMC_EINVAL, "geometry must be 0 or 1");
    if (!(s->fx > 0) || !(s->fy > 0) || !std::isfinite(s->fx) || !std::isfinite(s->fy))
        return fail(c, OMC_EINVAL, "field size must be > 0");
    if (s->geometry == 1 && !finite_pos(s->ssd)) return fail(c, OMC_EINVAL, "ssd must be > 0");
    const double chk[] = {s->z_field, s->cx, s->cy, s->sx, s->sy, s->gantry_deg, s->iso_x, s->iso_z};
    for (double v : chk)
        if (!std::isfinite(v)) return fail(c, OMC_EINVAL, "non-finite source geometry");
    std::vector<double> edges, weights, cdf;
    if (s->n_bins < 0 || s->n_bins > 4096) return fail(c, OMC_EINVAL, "n_bins out of range");
    if (s->n_bins == 0) {
        if (!(s->mono_E > 0) || !(s->mono_E < omc::kEHi))
            return fail(c, OMC_EINVAL, "mono_E must be in (0, 20) MeV");
    } else {
        if (!s->edges || !s->weights) return fail(c, OMC_EINVAL, "spectrum arrays are NULL");
        edges.assign(s->edges, s->edges + s->n_bins + 1);
        weights.assign(s->weights, s->weights + s->n_bins);
        for (int b = 0; b <= s->n_bins; ++b)
            if (!(edges[b] > 0) || !(edges[b] < omc::kEHi) || (b && !(edges[b] > edges[b - 1])))
                return fail(c, OMC_EINVAL, "spectrum edges must increase within (0, 20) MeV");
        double acc = 0.0;
        for (int b = 0; b < s->n_bins; ++b) {
            if (!(weights[b] >= 0) || !std::isfinite(weights[b]))
                return fail(c, OMC_EINVAL, "spectrum weights must be finite and >= 0");
            acc += weights[b];
            cdf.push_back(acc);
        }
        if (!(acc > 0)) return fail(c, OMC_EINVAL, "empty spectrum");
        for (double& v : cdf) v = v / acc;
    }
    dfree(c->d_cdf);
    if (!cdf.empty()) {
        if (hipMalloc(&c->d_cdf, cdf.size() * sizeof(double)) != hipSuccess)
            return fail(c, OMC_ENOMEM, "hipMalloc failed for the spectrum");
        HIP_TRY(c, hipMemcpy(c->d_cdf, cdf.data(), cdf.size() * sizeof(double),
                             hipMemcpyHostToDevice));
    }
    c->src = *s;
    c->edges = edges;
    c->weights = weights;
    c->cdf = cdf;
    c->src.edges = nullptr;
    c->src.weights = nullptr;
    dfree(c->t32.edges);
    dfree(c->t64.edges);
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
        p->queue_factor > 64 || p->chunk_histories < 0)
        return fail(c, OMC_EINVAL, "launch shape out of range");
    c->prm = *p;
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
    dfree(c->d_rho);
    dfree(c->d_mat);
    dfree(c->d_cdf);
    dfree(c->d_grid);
    dfree(c->d_dose);
    dfree(c->d_dose2);
    dfree(c->d_ctrl);
    dfree(c->d_counters);
    dfree(c->d_energies);
    if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
    delete c;
}

}  // extern "C"
