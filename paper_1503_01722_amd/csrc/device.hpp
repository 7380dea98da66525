// device.hpp -- gfx950 transport kernels, templated on the transport precision
// R (float for production, double for the parity build).
//
// Execution model (the paper's Table 1 and Sec. 2.2.1, re-shaped for CDNA4):
// the paper launches M work-items per iteration, all on particles of one type,
// picked from the photon stack, the electron stack or the source. Here each
// particle type has its own persistent kernel; every wave keeps 64 particles
// live and refills lanes whose particle ended from the input queue (ballot
// compaction), so a wave never idles on dead lanes while work remains.
// Secondaries are appended to the other queues with one atomic per wave
// (Sec. 2.2.2 uses one atomic per push). Dose goes to FP64 batch grids with
// hardware FP64 atomics (Sec. 2.2.2: atomic dose counter).
//
// Random numbers: Philox4x32-10 keyed by (seed, history), counter
// (block, id_lo, id_hi, 0); words of a block are used in order; a child's id is
// two words of its parent's stream (high bit set). Source particles use block 0
// of id 0 for sampling and continue at block 1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "engine.hpp"

namespace omc {

constexpr double kDevMC2 = 0.51099895;
constexpr double kDevPi = 3.14159265358979323846;
// Bounds on loops that end with probability one: rejection sampling (accept
// rates are above 1/3, so the bound is never reached in practice) and steps of
// one particle (a watchdog; a particle that reaches it leaves its energy where
// it stands and is counted).
constexpr int kMaxTries = 1000;
constexpr uint32_t kMaxSteps = 1u << 20;

// ---------------------------------------------------------------- math policy
template <typename R>
struct Math;

// Production: hardware transcendentals (v_log_f32 / v_exp_f32 / v_sin_f32 /
// v_rcp_f32 / v_sqrt_f32); about 1 ulp, ample for FP32 transport.
template <>
struct Math<float> {
    static __device__ __forceinline__ float log2(float x) { return __builtin_amdgcn_logf(x); }
    static __device__ __forceinline__ float log(float x)
    {
        return __builtin_amdgcn_logf(x) * 0.69314718055994531f;
    }
    static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
    static __device__ __forceinline__ float exp(float x)
    {
        return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
    }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float div(float a, float b)
    {
        return a * __builtin_amdgcn_rcpf(b);
    }
    // sin and cos of 2 pi u; v_sin_f32 / v_cos_f32 take revolutions
    static __device__ __forceinline__ void sincos_turns(float u, float& s, float& c)
    {
        s = __builtin_amdgcn_sinf(u);
        c = __builtin_amdgcn_cosf(u);
    }
    static __device__ __forceinline__ void sincos(float th, float& s, float& c)
    {
        s = __builtin_amdgcn_sinf(th * 0.15915494309189535f);
        c = __builtin_amdgcn_cosf(th * 0.15915494309189535f);
    }
    static __device__ __forceinline__ float floor(float x) { return __builtin_floorf(x); }
    static __device__ __forceinline__ float inf() { return __builtin_inff(); }
};

// Parity: IEEE double arithmetic in the same order as the CPU reference
// (compiled without FMA contraction), device-library transcendentals.
template <>
struct Math<double> {
    static __device__ __forceinline__ double log2(double x) { return ::log2(x); }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double exp2(double x) { return ::exp2(x); }
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ void sincos_turns(double u, double& s, double& c)
    {
        const double phi = (2.0 * kDevPi) * u;
        s = ::sin(phi);
        c = ::cos(phi);
    }
    static __device__ __forceinline__ void sincos(double th, double& s, double& c)
    {
        s = ::sin(th);
        c = ::cos(th);
    }
    static __device__ __forceinline__ double floor(double x) { return ::floor(x); }
    static __device__ __forceinline__ double inf() { return __builtin_inf(); }
};

template <typename R>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};

// ---------------------------------------------------------------- Philox
struct Stream {
    uint32_t k0, k1;   // seed, history
    uint32_t q0, q1;   // particle id
    uint32_t n;        // next block
    uint32_t w0, w1, w2, w3;
    uint32_t left;     // unused words of the cached block

    __device__ __forceinline__ void init(uint32_t seed, uint32_t h, uint32_t qlo, uint32_t qhi,
                                         uint32_t n0)
    {
        k0 = seed;
        k1 = h;
        q0 = qlo;
        q1 = qhi;
        n = n0;
        left = 0;
    }

    static __device__ __forceinline__ void block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t key0, uint32_t key1, uint32_t& o0,
                                                 uint32_t& o1, uint32_t& o2, uint32_t& o3)
    {
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const uint32_t lo0 = 0xD2511F53u * c0;
            const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
            const uint32_t lo1 = 0xCD9E8D57u * c2;
            const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
            const uint32_t n0 = hi1 ^ c1 ^ key0;
            const uint32_t n2 = hi0 ^ c3 ^ key1;
            c0 = n0;
            c1 = lo1;
            c2 = n2;
            c3 = lo0;
            key0 += 0x9E3779B9u;
            key1 += 0xBB67AE85u;
        }
        o0 = c0;
        o1 = c1;
        o2 = c2;
        o3 = c3;
    }

    __device__ __forceinline__ uint32_t word()
    {
        if (left == 0) {
            block(n, q0, q1, 0u, k0, k1, w0, w1, w2, w3);
            n += 1;
            left = 4;
        }
        const uint32_t out = w0;
        w0 = w1;
        w1 = w2;
        w2 = w3;
        left -= 1;
        return out;
    }

    // (2 (x >> 9) + 1) 2^-24: exact in float and double, never 0 or 1
    template <typename R>
    __device__ __forceinline__ R uniform()
    {
        const uint32_t x = word();
        return R(((x >> 9) << 1) | 1u) * R(5.9604644775390625e-08);
    }
};

// ---------------------------------------------------------------- particles
template <typename R>
struct Particle {
    R x, y, z, u, v, w, E;
    int ix, iy, iz;
    R nmfp;          // remaining hard-event mean free paths; < 0 unset
    int type;
    uint32_t h;      // history
    uint32_t batch;  // tally batch of the history
    Stream rng;
};

struct LaneStats {
    uint32_t c[kNumCounters];
    double e_dep, e_esc, e_inc;
    uint32_t max_steps;  // longest particle handled by the lane
};

__device__ __forceinline__ uint32_t pack_vox(int ix, int iy, int iz)
{
    return uint32_t(ix) | (uint32_t(iy) << 10) | (uint32_t(iz) << 20);
}

// ------------------------------------------------------------ wave primitives
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below()
{
    return (uint64_t(1) << lane_id()) - 1;
}

// Slot in q for each active lane that calls this together: one atomic per wave.
template <typename R>
__device__ __forceinline__ uint32_t wave_reserve(const QueueView<R>& q)
{
    const uint64_t active = __ballot(1);
    const int leader = __ffsll((unsigned long long)active) - 1;
    const uint32_t rank = __popcll(active & lanes_below());
    uint32_t base = 0;
    if (int(lane_id()) == leader) base = atomicAdd(q.count, uint32_t(__popcll(active)));
    base = __shfl(base, leader);
    return base + rank;
}

// ----------------------------------------------------------------- context
template <typename R>
struct Ctx {
    const KernelArgs<R>& a;
    // LDS-staged tables
    const typename Vec4<R>::type* ph;  // photon per material
    const R* muhat;
    const typename Vec4<R>::type* el;  // electron per material
    const R* K1;
    const R* msA;
    const R* Rabs;
    LaneStats& st;

    __device__ __forceinline__ size_t lin(int ix, int iy, int iz) const
    {
        return size_t(ix) + size_t(a.ph.nx) * (size_t(iy) + size_t(a.ph.ny) * size_t(iz));
    }

    __device__ __forceinline__ void deposit(const Particle<R>& p, size_t v, double e) const
    {
        unsafeAtomicAdd(&a.tally.grid[size_t(p.batch) * a.tally.nvox + v], e);
        st.e_dep += e;
    }
    // rounding residual of an energy split in the transport precision
    __device__ __forceinline__ void residual(const Particle<R>& p, size_t v, double e) const
    {
        if (e != 0.0) deposit(p, v, e);
    }

    // energy grid position: t = (log2 E - L0) * INV clamped to [0, NE-1]
    __device__ __forceinline__ void epos(R E, int& i, R& f) const
    {
        R t = (Math<R>::log2(E) - a.tab.L0) * a.tab.INV;
        if (t < R(0)) t = R(0);
        if (t > R(kTabNE - 1)) t = R(kTabNE - 1);
        i = int(Math<R>::floor(t));
        if (i > kTabNE - 2) i = kTabNE - 2;
        if (i < 0) i = 0;  // NaN input
        f = t - R(i);
    }

    static __device__ __forceinline__ R lerp(R y0, R y1, R f) { return y0 + f * (y1 - y0); }

    __device__ __forceinline__ R range_at(int m, R E) const
    {
        int i;
        R f;
        epos(E, i, f);
        const auto* t = el + m * kTabNE;
        return lerp(t[i].x, t[i + 1].x, f);
    }

    // exact inverse of the piecewise-linear range interpolant
    __device__ __forceinline__ R range_inverse(int m, R Rv) const
    {
        const auto* t = el + m * kTabNE;
        if (Rv <= t[0].x) return a.tab.ELo;
        if (Rv >= t[kTabNE - 1].x) return a.tab.EHi;
        int lo = 0, hi = kTabNE - 1;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (t[mid].x <= Rv) lo = mid;
            else hi = mid;
        }
        const R f = Math<R>::div(Rv - t[lo].x, t[lo + 1].x - t[lo].x);
        return Math<R>::exp2(a.tab.L0 + (R(lo) + f) * a.tab.DL);
    }

    __device__ __forceinline__ R screening(R x) const
    {
        R lx = Math<R>::log2(x);
        if (lx < a.tab.XLO) lx = a.tab.XLO;
        if (lx > a.tab.XHI) lx = a.tab.XHI;
        const R t = (lx - a.tab.XLO) * a.tab.XINV;
        int i = int(Math<R>::floor(t));
        if (i > kTabNA - 2) i = kTabNA - 2;
        if (i < 0) i = 0;  // NaN input
        const R f = t - R(i);
        return Math<R>::exp2(lerp(msA[i], msA[i + 1], f));
    }

    // ---- step trace of one history: code, particle id, stream position,
    // position, direction, energy, packed voxel (after the step)
    __device__ __forceinline__ void trace(const Particle<R>& p, int code) const
    {
        if (!a.trace.on || p.h != a.trace.h) return;
        const uint32_t k = atomicAdd(a.trace.n, 1u);
        if (k >= a.trace.cap) return;
        double* r = a.trace.buf + size_t(k) * kTraceWords;
        r[0] = code;
        r[1] = p.rng.q0;
        r[2] = p.rng.q1;
        r[3] = 4.0 * double(p.rng.n) - double(p.rng.left);
        r[4] = double(p.x);
        r[5] = double(p.y);
        r[6] = double(p.z);
        r[7] = double(p.u);
        r[8] = double(p.v);
        r[9] = double(p.w);
        r[10] = double(p.E);
        r[11] = double(p.ix) + 1024.0 * (double(p.iy) + 1024.0 * double(p.iz));
    }

    // ---- geometry
    __device__ __forceinline__ R coord(R x, R h, R ih) const
    {
        if constexpr (sizeof(R) == 8) return Math<R>::floor(x / h);
        else return Math<R>::floor(x * ih);
    }

    __device__ __forceinline__ bool locate(Particle<R>& p) const
    {
        const R fx = coord(p.x, a.ph.hx, a.ph.ihx);
        const R fy = coord(p.y, a.ph.hy, a.ph.ihy);
        const R fz = coord(p.z, a.ph.hz, a.ph.ihz);
        // written so that a NaN coordinate counts as outside
        if (!(fx >= R(0) && fx < R(a.ph.nx))) return false;
        if (!(fy >= R(0) && fy < R(a.ph.ny))) return false;
        if (!(fz >= R(0) && fz < R(a.ph.nz))) return false;
        p.ix = int(fx);
        p.iy = int(fy);
        p.iz = int(fz);
        return true;
    }

    // distance to the nearest face of the current voxel along (u,v,w);
    // ties go to the lower axis (x < y < z)
    __device__ __forceinline__ R dist_to_face(const Particle<R>& p, int& axis) const
    {
        R best = Math<R>::inf();
        axis = 0;
        const R pos[3] = {p.x, p.y, p.z};
        const R dir[3] = {p.u, p.v, p.w};
        const int idx[3] = {p.ix, p.iy, p.iz};
        const R hh[3] = {a.ph.hx, a.ph.hy, a.ph.hz};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            R s;
            if (dir[k] > R(0)) s = Math<R>::div(R(idx[k] + 1) * hh[k] - pos[k], dir[k]);
            else if (dir[k] < R(0)) s = Math<R>::div(R(idx[k]) * hh[k] - pos[k], dir[k]);
            else continue;
            if (s < best) {
                best = s;
                axis = k;
            }
        }
        if (best < R(0)) best = R(0);
        return best;
    }

    // ---- secondaries
    __device__ __forceinline__ void push(const QueueView<R>& q, const Particle<R>& p, int type, R E, R u, R v,
                         R w, uint32_t qlo, uint32_t qhi) const
    {
        const uint32_t slot = wave_reserve(q);
        if (slot >= q.cap) {
            atomicOr(a.stats.overflow, 1u);
            return;
        }
        q.x[slot] = p.x;
        q.y[slot] = p.y;
        q.z[slot] = p.z;
        q.u[slot] = u;
        q.v[slot] = v;
        q.w[slot] = w;
        q.E[slot] = E;
        q.vox[slot] = pack_vox(p.ix, p.iy, p.iz);
        q.hist[slot] = p.h;
        q.qlo[slot] = qlo;
        q.qhi[slot] = qhi;
        q.type[slot] = uint8_t(type);
    }

    __device__ __forceinline__ void emit_photon(Particle<R>& parent, R E, R u, R v, R w) const
    {
        if (E >= a.prm.Eabs_g) {
            const uint32_t lo = parent.rng.word();
            const uint32_t hi = parent.rng.word() | 0x80000000u;
            push(a.qp_out, parent, PT_PHOTON, E, u, v, w, lo, hi);
            st.c[C_PUSH_PH] += 1;
        } else {
            deposit(parent, lin(parent.ix, parent.iy, parent.iz), double(E));
        }
    }

    __device__ __forceinline__ void annihilate(Particle<R>& p) const
    {
        st.c[C_POS_ANNIHIL] += 1;
        const R c = R(2) * p.rng.template uniform<R>() - R(1);
        R sp, cp;
        Math<R>::sincos_turns(p.rng.template uniform<R>(), sp, cp);
        const R s = Math<R>::sqrt((R(1) - c) * (R(1) + c));
        const R ax = s * cp, ay = s * sp, az = c;
        const R m = R(kDevMC2);
        // the two photons carry the transport-precision rest energy
        residual(p, lin(p.ix, p.iy, p.iz), 2.0 * kDevMC2 - 2.0 * double(m));
        emit_photon(p, m, ax, ay, az);
        emit_photon(p, m, -ax, -ay, -az);
    }

    __device__ __forceinline__ void emit_electron(Particle<R>& parent, int type, R E, R u, R v, R w) const
    {
        if (!a.prm.kerma && E >= a.prm.Eabs_e) {
            const uint32_t lo = parent.rng.word();
            const uint32_t hi = parent.rng.word() | 0x80000000u;
            push(a.qe_out, parent, type, E, u, v, w, lo, hi);
            st.c[C_PUSH_EL] += 1;
        } else {
            deposit(parent, lin(parent.ix, parent.iy, parent.iz), double(E));
            if (type == PT_POSITRON) annihilate(parent);
        }
    }

    static __device__ __forceinline__ void rotate(R& u, R& v, R& w, R cost, R sint, R cphi, R sphi)
    {
        const R r2 = R(1) - w * w;
        if (r2 < R(1e-12)) {
            u = sint * cphi;
            v = sint * sphi;
            w = w >= R(0) ? cost : -cost;
            return;
        }
        const R r = Math<R>::sqrt(r2);
        const R nu = u * cost + Math<R>::div(sint * (u * w * cphi - v * sphi), r);
        const R nv = v * cost + Math<R>::div(sint * (v * w * cphi + u * sphi), r);
        const R nw = w * cost - sint * cphi * r;
        u = nu;
        v = nv;
        w = nw;
    }

    // ---- photons (Sec. 2.1)
    __device__ __forceinline__ void compton(Particle<R>& p) const
    {
        const R E = p.E;
        const R k = Math<R>::div(E, R(kDevMC2));
        const R e0 = Math<R>::div(R(1), R(1) + R(2) * k);
        const R a1 = Math<R>::log(R(1) + R(2) * k);
        const R a2 = R(0.5) * (R(1) - e0 * e0);
        R eps, t;
        for (int tries = 0;; ++tries) {
            const R ua = p.rng.template uniform<R>();
            const R ub = p.rng.template uniform<R>();
            const R uc = p.rng.template uniform<R>();
            if (ua * (a1 + a2) < a1) eps = Math<R>::exp(-a1 * ub);
            else eps = Math<R>::sqrt(e0 * e0 + (R(1) - e0 * e0) * ub);
            t = Math<R>::div(R(1) - eps, k * eps);
            const R sin2 = t * (R(2) - t);
            if (uc <= R(1) - Math<R>::div(eps * sin2, R(1) + eps * eps) || tries >= kMaxTries)
                break;
        }
        const R sin2 = t * (R(2) - t);
        const R cost = R(1) - t;
        const R sint = Math<R>::sqrt(sin2 > R(0) ? sin2 : R(0));
        R sf, cf;
        Math<R>::sincos_turns(p.rng.template uniform<R>(), sf, cf);
        const R u0 = p.u, v0 = p.v, w0 = p.w;
        rotate(p.u, p.v, p.w, cost, sint, cf, sf);
        const R Ep = eps * E;
        const R Te = E - Ep;
        const R px = E * u0 - Ep * p.u, py = E * v0 - Ep * p.v, pz = E * w0 - Ep * p.w;
        const R nrm = Math<R>::sqrt(px * px + py * py + pz * pz);
        R eu = u0, ev = v0, ew = w0;
        if (nrm > R(0)) {
            eu = Math<R>::div(px, nrm);
            ev = Math<R>::div(py, nrm);
            ew = Math<R>::div(pz, nrm);
        }
        st.c[C_PH_COMPTON] += 1;
        residual(p, lin(p.ix, p.iy, p.iz), double(E) - double(Ep) - double(Te));
        emit_electron(p, PT_ELECTRON, Te, eu, ev, ew);
        p.E = Ep;
    }

    __device__ __forceinline__ void pair(Particle<R>& p) const
    {
        const R K = p.E - R(2.0 * kDevMC2);
        const R Tm = p.rng.template uniform<R>() * K;
        const R Tp = K - Tm;
        st.c[C_PH_PAIR] += 1;
        residual(p, lin(p.ix, p.iy, p.iz),
                 double(p.E) - 2.0 * kDevMC2 - double(Tm) - double(Tp));
        emit_electron(p, PT_ELECTRON, Tm, p.u, p.v, p.w);
        emit_electron(p, PT_POSITRON, Tp, p.u, p.v, p.w);
    }

    // One Woodcock flight and, if real, the interaction. false = photon ended.
    __device__ __forceinline__ bool photon_step(Particle<R>& p) const
    {
        if (p.E < a.prm.Eabs_g) {
            deposit(p, lin(p.ix, p.iy, p.iz), double(p.E));
            st.c[C_PH_CUTOFF] += 1;
            return false;
        }
        int i;
        R f;
        epos(p.E, i, f);
        const R mh = lerp(muhat[i], muhat[i + 1], f);
        const R s = Math<R>::div(-Math<R>::log(p.rng.template uniform<R>()), mh);
        p.x = p.x + s * p.u;
        p.y = p.y + s * p.v;
        p.z = p.z + s * p.w;
        st.c[C_PH_FLIGHTS] += 1;
        if (!locate(p)) {
            st.e_esc += double(p.E);
            st.c[C_PH_ESCAPED] += 1;
            return false;
        }
        const size_t vx = lin(p.ix, p.iy, p.iz);
        const int m = a.ph.mat[vx];
        const R rho = R(a.ph.rho[vx]);
        const auto* t = ph + m * kTabNE;
        const auto n0 = t[i], n1 = t[i + 1];
        const R mt = lerp(n0.x, n1.x, f);
        if (!(p.rng.template uniform<R>() * mh < rho * mt)) {
            st.c[C_PH_FICT] += 1;
            return true;
        }
        const R sel = p.rng.template uniform<R>() * mt;
        const R mc = lerp(n0.y, n1.y, f);
        const R mp = lerp(n0.z, n1.z, f);
        if (sel < mc) {
            compton(p);
            return true;
        }
        if (sel < mc + mp || p.E <= R(2.0 * kDevMC2)) {
            deposit(p, vx, double(p.E));
            st.c[C_PH_PHOTO] += 1;
            return false;
        }
        pair(p);
        return false;
    }

    // ---- electrons and positrons (Sec. 2.1, Class II condensed history)
    __device__ __forceinline__ void moller(Particle<R>& p, size_t vx) const
    {
        const R T = p.E;
        if (!(T > R(2) * a.prm.Wcc)) {
            st.c[C_EL_HARD_FICT] += 1;
            return;
        }
        const R e0 = Math<R>::div(a.prm.Wcc, T);
        const R tau = Math<R>::div(T, R(kDevMC2));
        const R g = tau + R(1);
        const R aa = Math<R>::div(tau, g);
        const R bb = Math<R>::div(R(2) * tau + R(1), g * g);
        R eps;
        for (int tries = 0;; ++tries) {
            const R ua = p.rng.template uniform<R>();
            const R ub = p.rng.template uniform<R>();
            eps = Math<R>::div(e0, R(1) - ua * (R(1) - R(2) * e0));
            const R rr = Math<R>::div(eps, R(1) - eps);
            if (ub * (R(2) + R(0.25) * aa * aa) <= R(1) + rr * rr + aa * aa * eps * eps - bb * rr ||
                tries >= kMaxTries)
                break;
        }
        const R W = eps * T;
        const R Tp = T - W;
        const R m2 = R(2.0 * kDevMC2);
        const R cp = Math<R>::sqrt(Math<R>::div(Tp * (T + m2), T * (Tp + m2)));
        const R cd = Math<R>::sqrt(Math<R>::div(W * (T + m2), T * (W + m2)));
        const R sp = Math<R>::sqrt(R(1) - cp * cp > R(0) ? R(1) - cp * cp : R(0));
        const R sd = Math<R>::sqrt(R(1) - cd * cd > R(0) ? R(1) - cd * cd : R(0));
        R sf, cf;
        Math<R>::sincos_turns(p.rng.template uniform<R>(), sf, cf);
        R du = p.u, dv = p.v, dw = p.w;
        rotate(du, dv, dw, cd, sd, -cf, -sf);  // delta at azimuth phi + pi
        rotate(p.u, p.v, p.w, cp, sp, cf, sf);
        st.c[C_EL_MOLLER] += 1;
        residual(p, vx, double(T) - double(Tp) - double(W));
        p.E = Tp;
        emit_electron(p, PT_ELECTRON, W, du, dv, dw);
    }

    __device__ __forceinline__ void brems(Particle<R>& p, size_t vx) const
    {
        const R T = p.E;
        if (!(T > a.prm.kc)) {
            st.c[C_EL_HARD_FICT] += 1;
            return;
        }
        const R lr = Math<R>::log(Math<R>::div(T, a.prm.kc));
        R k;
        for (int tries = 0;; ++tries) {
            const R ua = p.rng.template uniform<R>();
            const R ub = p.rng.template uniform<R>();
            k = a.prm.kc * Math<R>::exp(ua * lr);
            const R y = Math<R>::div(k, T);
            if (ub <= R(1) - y + R(0.75) * y * y || tries >= kMaxTries) break;
        }
        const R th = Math<R>::div(R(kDevMC2), T + R(kDevMC2));
        R st_, ct_;
        Math<R>::sincos(th, st_, ct_);
        R sf, cf;
        Math<R>::sincos_turns(p.rng.template uniform<R>(), sf, cf);
        R gu = p.u, gv = p.v, gw = p.w;
        rotate(gu, gv, gw, ct_, st_, cf, sf);
        st.c[C_EL_BREMS] += 1;
        const R Tn = T - k;
        residual(p, vx, double(T) - double(Tn) - double(k));
        p.E = Tn;
        emit_photon(p, k, gu, gv, gw);
    }

    __device__ __forceinline__ void hard_event(Particle<R>& p, int m, R shm, size_t vx) const
    {
        st.c[C_EL_HARD_CAND] += 1;
        int i;
        R f;
        epos(p.E, i, f);
        const auto* t = el + m * kTabNE;
        const R sM = lerp(t[i].z, t[i + 1].z, f);
        const R sB = lerp(t[i].w, t[i + 1].w, f);
        const R sH = sM + sB;
        if (p.rng.template uniform<R>() * shm < sH) {
            if (p.rng.template uniform<R>() * sH < sM) moller(p, vx);
            else brems(p, vx);
        } else {
            st.c[C_EL_HARD_FICT] += 1;
        }
        p.nmfp = -Math<R>::log(p.rng.template uniform<R>());
    }

    // One condensed-history step. false = particle ended.
    __device__ __forceinline__ bool electron_step(Particle<R>& p) const
    {
        const size_t vx = lin(p.ix, p.iy, p.iz);
        if (p.E <= a.prm.Eabs_e) {
            deposit(p, vx, double(p.E));
            st.c[C_EL_ABSORBED] += 1;
            trace(p, 64);
            if (p.type == PT_POSITRON) annihilate(p);
            return false;
        }
        const int m = a.ph.mat[vx];
        const R rho = R(a.ph.rho[vx]);
        const bool csda = a.prm.csda != 0;
        if (!csda && p.nmfp < R(0)) p.nmfp = -Math<R>::log(p.rng.template uniform<R>());
        const R T0 = p.E;
        int i;
        R f;
        epos(T0, i, f);
        const auto* t = el + m * kTabNE;
        const R RT = lerp(t[i].x, t[i + 1].x, f);
        const R shm = lerp(t[i].y, t[i + 1].y, f);
        const R sig_hat = rho * shm;
        R d_event = Math<R>::inf();
        if (!csda && sig_hat > R(0)) d_event = Math<R>::div(p.nmfp, sig_hat);
        int ax;
        const R d_vox = dist_to_face(p, ax);
        const R d_maxs = a.prm.dmax_s;
        const R d_maxe = Math<R>::div(RT - range_at(m, a.prm.one_minus_fE * T0), rho);
        const R d_abs = Math<R>::div(RT - Rabs[m], rho);
        enum { VOX = 0, MAXS, MAXE, ABS, EVENT };
        R d = d_vox;
        int lim = VOX;
        if (d_maxs < d) { d = d_maxs; lim = MAXS; }
        if (d_maxe < d) { d = d_maxe; lim = MAXE; }
        if (d_abs < d) { d = d_abs; lim = ABS; }
        if (d_event < d) { d = d_event; lim = EVENT; }

        bool crossed = false;
        int cax = ax;
        if (d > R(0)) {
            R s;
            // straight line in CSDA mode, and inside the boundary skin where the
            // hinge deflection is skipped so that the step ends on the face
            if (csda || (lim == VOX && d < a.prm.skin)) {
                p.x = p.x + d * p.u;
                p.y = p.y + d * p.v;
                p.z = p.z + d * p.w;
                s = d;
                crossed = lim == VOX;
            } else {
                // random hinge: straight to xi*d, deflect, then the remainder
                const R xi = p.rng.template uniform<R>();
                const R s1 = xi * d;
                p.x = p.x + s1 * p.u;
                p.y = p.y + s1 * p.v;
                p.z = p.z + s1 * p.w;
                const R Tplan = range_inverse(m, RT - rho * d);
                const R Tmid = R(0.5) * (T0 + Tplan);
                int i2;
                R f2;
                epos(Tmid, i2, f2);
                const R k1 = lerp(K1[m * kTabNE + i2], K1[m * kTabNE + i2 + 1], f2);
                const R A = screening(d * rho * k1);
                const R um = p.rng.template uniform<R>();
                R omc = Math<R>::div(R(2) * A * um, R(1) + A - um);
                if (omc > R(2)) omc = R(2);  // rounding of the fast reciprocal (FP32)
                R sf, cf;
                Math<R>::sincos_turns(p.rng.template uniform<R>(), sf, cf);
                rotate(p.u, p.v, p.w, R(1) - omc, Math<R>::sqrt(omc * (R(2) - omc)), cf, sf);
                const R rem = (R(1) - xi) * d;
                int ax2;
                const R dv2 = dist_to_face(p, ax2);
                R s2 = rem;
                if (dv2 < rem) {
                    s2 = dv2;
                    crossed = true;
                    cax = ax2;
                    st.c[C_EL_HINGE_TRUNC] += 1;
                }
                p.x = p.x + s2 * p.u;
                p.y = p.y + s2 * p.v;
                p.z = p.z + s2 * p.w;
                s = s1 + s2;
            }
            R Tend;
            if (lim == ABS && !crossed) Tend = a.prm.Eabs_e;
            else Tend = range_inverse(m, RT - rho * s);
            deposit(p, vx, double(T0) - double(Tend));
            if (!csda) {
                p.nmfp = p.nmfp - sig_hat * s;
                if (p.nmfp < R(0)) p.nmfp = R(0);
            }
            st.c[C_EL_STEPS] += 1;
            p.E = Tend;
        } else if (lim == VOX) {
            crossed = true;  // zero-length step on a face: only the index moves
        } else if (lim == ABS) {
            // no range left above the absorption energy (T within rounding of
            // E_abs): the track ends; the remainder is deposited here
            deposit(p, vx, double(T0) - double(a.prm.Eabs_e));
            p.E = a.prm.Eabs_e;
        }

        if (crossed) {
            // snap onto the face and step the index (no re-flooring)
            bool out;
            if (cax == 0) {
                const bool up = p.u > R(0);
                p.x = up ? R(p.ix + 1) * a.ph.hx : R(p.ix) * a.ph.hx;
                p.ix += up ? 1 : -1;
                out = p.ix < 0 || p.ix >= a.ph.nx;
            } else if (cax == 1) {
                const bool up = p.v > R(0);
                p.y = up ? R(p.iy + 1) * a.ph.hy : R(p.iy) * a.ph.hy;
                p.iy += up ? 1 : -1;
                out = p.iy < 0 || p.iy >= a.ph.ny;
            } else {
                const bool up = p.w > R(0);
                p.z = up ? R(p.iz + 1) * a.ph.hz : R(p.iz) * a.ph.hz;
                p.iz += up ? 1 : -1;
                out = p.iz < 0 || p.iz >= a.ph.nz;
            }
            st.c[C_EL_BOUNDARY] += 1;
            trace(p, 16 + lim + 8 * int(crossed));
            if (out) {
                st.e_esc += double(p.E);
                st.c[C_EL_ESCAPED] += 1;
                return false;
            }
            return true;
        }
        if (lim == EVENT) hard_event(p, m, shm, vx);
        trace(p, 16 + lim);
        return true;
    }
};

// ------------------------------------------------------------- LDS staging
template <typename T>
__device__ __forceinline__ void stage(T* dst, const T* src, size_t n)
{
    for (size_t k = threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
}

// Wave-level sum of a per-lane value, added once per wave.
__device__ __forceinline__ void wave_flush_u64(unsigned long long* dst, uint32_t v)
{
    unsigned long long s = v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane_id() == 0 && s) atomicAdd(dst, s);
}

__device__ __forceinline__ void wave_flush_f64(double* dst, double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane_id() == 0 && v != 0.0) unsafeAtomicAdd(dst, v);
}

__device__ __forceinline__ void flush_stats(const StatsView& sv, const LaneStats& st)
{
#pragma unroll
    for (int k = 0; k < kNumCounters; ++k) wave_flush_u64(&sv.counters[k], st.c[k]);
    wave_flush_f64(&sv.energies[EN_DEPOSITED], st.e_dep);
    wave_flush_f64(&sv.energies[EN_ESCAPED], st.e_esc);
    wave_flush_f64(&sv.energies[EN_INCIDENT], st.e_inc);
    uint32_t m = st.max_steps;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, uint32_t(__shfl_xor(m, off)));
    if (lane_id() == 0 && m) atomicMax(sv.max_steps, m);
}

__device__ __forceinline__ uint32_t batch_of(const TallyView& t, uint32_t h)
{
    return uint32_t((uint64_t(h - t.h0) * uint64_t(t.B)) / t.n_total);
}

template <typename R>
__device__ __forceinline__ void load_particle(const KernelArgs<R>& a, uint32_t slot,
                                              Particle<R>& p)
{
    const QueueView<R>& q = a.qin;
    p.x = q.x[slot];
    p.y = q.y[slot];
    p.z = q.z[slot];
    p.u = q.u[slot];
    p.v = q.v[slot];
    p.w = q.w[slot];
    p.E = q.E[slot];
    const uint32_t vp = q.vox[slot];
    p.ix = int(vp & 1023u);
    p.iy = int((vp >> 10) & 1023u);
    p.iz = int(vp >> 20);
    p.h = q.hist[slot];
    const uint32_t qlo = q.qlo[slot], qhi = q.qhi[slot];
    p.type = q.type[slot];
    p.nmfp = R(-1);
    p.batch = batch_of(a.tally, p.h);
    // the source particle (id 0) used block 0 for its sampling
    p.rng.init(a.seed, p.h, qlo, qhi, (qlo | qhi) == 0u ? 1u : 0u);
}

// ------------------------------------------------------------ transport loop
// Persistent wave loop: lanes whose particle ended take the next records of the
// wave's chunk of the input queue; a new chunk is claimed with one atomic.
template <typename R, bool kPhoton>
__device__ __forceinline__ void transport_loop(const KernelArgs<R>& a, const Ctx<R>& cx)
{
    const uint32_t n_in = *a.qin.count < a.qin.cap ? *a.qin.count : a.qin.cap;
    Particle<R> p;
    bool alive = false;
    uint32_t steps = 0;
    uint32_t pos = 0, end = 0;  // wave-uniform chunk window
    bool drained = false;
    for (;;) {
        uint64_t dead = __ballot(!alive);
        while (dead != 0 && !drained) {
            if (pos >= end) {
                uint32_t base = 0;
                if (lane_id() == 0) base = atomicAdd(a.qin.head, uint32_t(a.chunk));
                base = __shfl(base, 0);
                if (base >= n_in) {
                    drained = true;
                    break;
                }
                pos = base;
                end = base + uint32_t(a.chunk) < n_in ? base + uint32_t(a.chunk) : n_in;
            }
            const uint32_t avail = end - pos;
            const uint32_t rank = __popcll(dead & lanes_below());
            if (!alive && rank < avail) {
                load_particle(a, pos + rank, p);
                alive = true;
                steps = 0;
            }
            const uint32_t ndead = __popcll(dead);
            pos += ndead < avail ? ndead : avail;
            dead = __ballot(!alive);
        }
        if (__ballot(alive) == 0) break;
        if (alive) {
            alive = kPhoton ? cx.photon_step(p) : cx.electron_step(p);
            ++steps;
            if (alive && steps >= kMaxSteps) {
                cx.deposit(p, cx.lin(p.ix, p.iy, p.iz), double(p.E));
                cx.st.c[C_WATCHDOG] += 1;
                alive = false;
            }
            if (!alive && steps > cx.st.max_steps) cx.st.max_steps = steps;
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(256) photon_kernel(KernelArgs<R> a)
{
    using V4 = typename Vec4<R>::type;
    extern __shared__ __align__(32) unsigned char smem[];
    const int nm = a.tab.n_mats;
    V4* s_ph = reinterpret_cast<V4*>(smem);
    R* s_muhat = reinterpret_cast<R*>(s_ph + size_t(nm) * kTabNE);
    stage(s_ph, reinterpret_cast<const V4*>(a.tab.ph), size_t(nm) * kTabNE);
    stage(s_muhat, a.tab.muhat, size_t(kTabNE));
    __syncthreads();
    LaneStats st{};
    const Ctx<R> cx{a, s_ph, s_muhat, nullptr, nullptr, nullptr, nullptr, st};
    transport_loop<R, true>(a, cx);
    flush_stats(a.stats, st);
}

template <typename R>
__global__ void __launch_bounds__(256) electron_kernel(KernelArgs<R> a)
{
    using V4 = typename Vec4<R>::type;
    extern __shared__ __align__(32) unsigned char smem[];
    const int nm = a.tab.n_mats;
    V4* s_el = reinterpret_cast<V4*>(smem);
    R* s_K1 = reinterpret_cast<R*>(s_el + size_t(nm) * kTabNE);
    R* s_msA = s_K1 + size_t(nm) * kTabNE;
    R* s_Rabs = s_msA + kTabNA;
    stage(s_el, reinterpret_cast<const V4*>(a.tab.el), size_t(nm) * kTabNE);
    stage(s_K1, a.tab.K1, size_t(nm) * kTabNE);
    stage(s_msA, a.tab.msA, size_t(kTabNA));
    stage(s_Rabs, a.tab.Rabs, size_t(nm));
    __syncthreads();
    LaneStats st{};
    const Ctx<R> cx{a, nullptr, nullptr, s_el, s_K1, s_msA, s_Rabs, st};
    transport_loop<R, false>(a, cx);
    flush_stats(a.stats, st);
}

// ------------------------------------------------------------------- source
// One work-item per history (Sec. 2.2 "Materials": point source at SSD,
// field at the phantom surface). Draws block 0 of (seed, h, id 0): u1, u2 for
// the energy, u3, u4 for the field point.
template <typename R>
__global__ void __launch_bounds__(256) source_kernel(KernelArgs<R> a)
{
    LaneStats st{};
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const Ctx<R> cx{a, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, st};
    if (i < a.src_count) {
        const SourceView<R>& S = a.src;
        Particle<R> p;
        p.h = a.tally.h0 + a.src_begin + i;
        p.batch = batch_of(a.tally, p.h);
        Stream r;
        r.init(a.seed, p.h, 0u, 0u, 0u);
        const double u1 = double(r.uniform<R>());
        const R u2 = r.uniform<R>(), u3 = r.uniform<R>(), u4 = r.uniform<R>();
        R E = S.mono_E;
        if (S.n_bins > 0) {
            int b = 0;
            while (b < S.n_bins - 1 && !(S.cdf[b] > u1)) ++b;
            E = S.edges[b] + u2 * (S.edges[b + 1] - S.edges[b]);
        }
        R X[3] = {S.cx + (u3 - R(0.5)) * S.fx, S.cy + (u4 - R(0.5)) * S.fy, S.z_field};
        R d[3] = {R(0), R(0), R(1)};
        R tS = -Math<R>::inf();
        if (S.point) {
            const R ex = X[0] - S.sx, ey = X[1] - S.sy, ez = X[2] - (S.z_field - S.ssd);
            const R nrm = Math<R>::sqrt(ex * ex + ey * ey + ez * ez);
            d[0] = Math<R>::div(ex, nrm);
            d[1] = Math<R>::div(ey, nrm);
            d[2] = Math<R>::div(ez, nrm);
            tS = -nrm;
        }
        if (S.rotate) {
            const R px = X[0] - S.iso_x, pz = X[2] - S.iso_z;
            X[0] = S.iso_x + S.cg * px + S.sg * pz;
            X[2] = S.iso_z - S.sg * px + S.cg * pz;
            const R dx = d[0], dz = d[2];
            d[0] = S.cg * dx + S.sg * dz;
            d[2] = -S.sg * dx + S.cg * dz;
        }
        R t0 = -Math<R>::inf(), t1 = Math<R>::inf();
        const R L[3] = {R(a.ph.nx) * a.ph.hx, R(a.ph.ny) * a.ph.hy, R(a.ph.nz) * a.ph.hz};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (d[k] != R(0)) {
                R ta = Math<R>::div(R(0) - X[k], d[k]);
                R tb = Math<R>::div(L[k] - X[k], d[k]);
                if (ta > tb) {
                    const R sw = ta;
                    ta = tb;
                    tb = sw;
                }
                if (ta > t0) t0 = ta;
                if (tb < t1) t1 = tb;
            } else if (X[k] < R(0) || X[k] >= L[k]) {
                t0 = Math<R>::inf();
            }
        }
        st.e_inc += double(E);
        if (!(t0 < t1) || t1 <= tS) {
            st.e_esc += double(E);
            st.c[C_SRC_MISS] += 1;
        } else {
            const R tt = t0 > tS ? t0 : tS;
            p.x = X[0] + tt * d[0];
            p.y = X[1] + tt * d[1];
            p.z = X[2] + tt * d[2];
            const R hh[3] = {a.ph.hx, a.ph.hy, a.ph.hz};
            const int nn[3] = {a.ph.nx, a.ph.ny, a.ph.nz};
            const R pp[3] = {p.x, p.y, p.z};
            int iv[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                R fl = cx.coord(pp[k], hh[k], R(1) / hh[k]);
                if (fl < R(0)) fl = R(0);
                if (fl > R(nn[k] - 1)) fl = R(nn[k] - 1);
                iv[k] = int(fl);
            }
            p.ix = iv[0];
            p.iy = iv[1];
            p.iz = iv[2];
            p.E = E;
            if (S.particle == 0) {
                cx.push(a.qp_out, p, PT_PHOTON, E, d[0], d[1], d[2], 0u, 0u);
            } else if (a.prm.kerma) {
                cx.deposit(p, cx.lin(p.ix, p.iy, p.iz), double(E));
            } else {
                cx.push(a.qe_out, p, PT_ELECTRON, E, d[0], d[1], d[2], 0u, 0u);
            }
        }
    }
    flush_stats(a.stats, st);
}

}  // namespace omc
