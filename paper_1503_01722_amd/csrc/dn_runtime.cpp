// dn_runtime.cpp -- the learned dose denoiser (include/omc_dn.h): U-Net
// wiring over the gfx950 kernels of dn_kernels.hip, training step, gradient,
// denoising with plain Monte Carlo as fallback, and the layer test entry.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/omc_dn.h"
#include "dn.hpp"
#include "engine.hpp"

namespace {

thread_local std::string g_dn_error;

constexpr int kLevels = 4;
constexpr int kChan[kLevels] = {16, 32, 48, 64};
constexpr int kInChannels = 3;
constexpr int kInPadded = 8;

enum Kind : int { K_CONV3 = 0, K_DOWN, K_UP, K_HEAD };

struct Layer {
    const char* name;
    int kind;
    int cin_log, cin, cout;
    int taps;
    size_t w_off = 0, b_off = 0;
    uint16_t* pk_fwd = nullptr;
    uint16_t* pk_bwd = nullptr;
    int Kf = 0, Nf = 0, Kb = 0, Nb = 0;
    bool need_bwd = true;
};

// [0] full resolution ... [3] 1/8
struct Level {
    dn::Dims d;
    size_t n;
};

}  // namespace

struct omc_dn {
    int device = 0;
    Level lv[kLevels];
    std::vector<Layer> layers;
    size_t n_params = 0;
    float* p = nullptr;   // master parameters
    float* gp = nullptr;  // gradient
    float* m = nullptr;
    float* v = nullptr;
    int step = 0;

    // activations (BF16) and their gradients (FP32)
    uint16_t* xin = nullptr;
    uint16_t* act[32] = {};
    float* grad[32] = {};
    uint16_t* scratch = nullptr;  // masked output gradient (BF16)
    float* y = nullptr;           // normalised output
    float* gy = nullptr;
    float* sums = nullptr;        // loss sums (device)
    float* h_sums = nullptr;      // pinned

    // denoise workspace
    double* d64 = nullptr;   // dose, dose2 (FP64, 2 volumes)
    float* f32 = nullptr;    // dose, sigma (FP32, 2 volumes)
    double* acc = nullptr;   // error sums (device, 8 doubles)
    double* h_acc = nullptr; // pinned

    std::vector<void*> allocs;
    std::string err;
};

namespace {

// activation slots
enum Slot : int {
    S_ENC1A = 0, S_ENC1B, S_DOWN2, S_ENC2A, S_ENC2B, S_DOWN3, S_ENC3A, S_ENC3B, S_DOWN4, S_ENC4A,
    S_ENC4B, S_UP3, S_DEC3A, S_DEC3B, S_UP2, S_DEC2A, S_DEC2B, S_UP1, S_DEC1A, S_DEC1B, S_COUNT
};

int dn_fail(omc_dn* d, int code, const std::string& msg)
{
    if (d) d->err = msg;
    g_dn_error = msg;
    return code;
}

template <typename T>
bool dalloc(omc_dn* d, T*& p, size_t n)
{
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return false;
    d->allocs.push_back(q);
    p = static_cast<T*>(q);
    return true;
}

// He-normal initial weights from a counter-based hash (splitmix64) and the
// Box-Muller transform; zero biases.
uint64_t splitmix(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

double normal_of(uint32_t seed, uint64_t i)
{
    const uint64_t a = splitmix((uint64_t(seed) << 40) ^ (2 * i));
    const uint64_t b = splitmix((uint64_t(seed) << 40) ^ (2 * i + 1));
    const double u1 = (double(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = double(b >> 11) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

void build_layers(omc_dn* d)
{
    const int c1 = kChan[0], c2 = kChan[1], c3 = kChan[2], c4 = kChan[3];
    auto L = [](const char* n, int kind, int cin_log, int cin, int cout) {
        Layer l;
        l.name = n;
        l.kind = kind;
        l.cin_log = cin_log;
        l.cin = cin;
        l.cout = cout;
        l.taps = kind == K_CONV3 ? 27 : kind == K_HEAD ? 1 : 8;
        return l;
    };
    d->layers = {L("enc1a", K_CONV3, kInChannels, kInPadded, c1), L("enc1b", K_CONV3, c1, c1, c1),
                 L("down2", K_DOWN, c1, c1, c2),   L("enc2a", K_CONV3, c2, c2, c2),
                 L("enc2b", K_CONV3, c2, c2, c2),  L("down3", K_DOWN, c2, c2, c3),
                 L("enc3a", K_CONV3, c3, c3, c3),  L("enc3b", K_CONV3, c3, c3, c3),
                 L("down4", K_DOWN, c3, c3, c4),   L("enc4a", K_CONV3, c4, c4, c4),
                 L("enc4b", K_CONV3, c4, c4, c4),  L("up3", K_UP, c4, c4, c3),
                 L("dec3a", K_CONV3, 2 * c3, 2 * c3, c3), L("dec3b", K_CONV3, c3, c3, c3),
                 L("up2", K_UP, c3, c3, c2),       L("dec2a", K_CONV3, 2 * c2, 2 * c2, c2),
                 L("dec2b", K_CONV3, c2, c2, c2),  L("up1", K_UP, c2, c2, c1),
                 L("dec1a", K_CONV3, 2 * c1, 2 * c1, c1), L("dec1b", K_CONV3, c1, c1, c1),
                 L("head", K_HEAD, c1, c1, 1)};
    d->layers[0].need_bwd = false;
    size_t at = 0;
    for (Layer& l : d->layers) {
        l.w_off = at;
        at += size_t(l.taps) * l.cin_log * l.cout;
        l.b_off = at;
        at += size_t(l.cout);
        switch (l.kind) {
        case K_CONV3:
            l.Kf = 27 * l.cin; l.Nf = l.cout; l.Kb = 27 * l.cout; l.Nb = l.cin; break;
        case K_DOWN:
            l.Kf = 8 * l.cin; l.Nf = l.cout; l.Kb = l.cout; l.Nb = 8 * l.cin; break;
        case K_UP:
            l.Kf = l.cin; l.Nf = 8 * l.cout; l.Kb = 8 * l.cout; l.Nb = l.cin; break;
        default: break;
        }
    }
    d->n_params = at;
}

int repack(omc_dn* d, hipStream_t s)
{
    for (Layer& l : d->layers) {
        if (l.kind == K_HEAD) continue;
        const float* w = d->p + l.w_off;
        const int fm = l.kind == K_UP ? dn::PACK_FWD_UP : dn::PACK_FWD;
        if (dn::launch_pack(w, l.taps, l.cin_log, l.cin, l.cout, fm, l.pk_fwd, s))
            return dn_fail(d, OMC_EDEVICE, "weight packing launch failed");
        if (!l.need_bwd) continue;
        const int bm = l.kind == K_CONV3 ? dn::PACK_BWD_FLIP
                       : l.kind == K_UP  ? dn::PACK_BWD
                                         : dn::PACK_BWD_UP;
        if (dn::launch_pack(w, l.taps, l.cin_log, l.cin, l.cout, bm, l.pk_bwd, s))
            return dn_fail(d, OMC_EDEVICE, "weight packing launch failed");
    }
    return OMC_OK;
}

const Layer& layer(const omc_dn* d, int i) { return d->layers[size_t(i)]; }

// forward pass from the packed input xin; leaves every activation in place
int forward_pass(omc_dn* d, const float* dose, const float* sigma, const float* rho, float inv_dmax,
                 float* out, hipStream_t s)
{
    const Level* L = d->lv;
    const size_t n = L[0].n;
    if (dn::launch_pack_input(dose, sigma, rho, inv_dmax, n, d->xin, s))
        return dn_fail(d, OMC_EDEVICE, "input packing launch failed");
    auto conv = [&](int li, int geometry, const uint16_t* x0, int c0, const uint16_t* x1, int c1,
                    int lin, int lout, int slot) {
        const Layer& l = layer(d, li);
        dn::ConvOut o;
        o.y = d->act[slot];
        o.bias = d->p + l.b_off;
        o.relu = 1;
        return dn::launch_conv(geometry, x0, c0, x1, c1, L[lin].d, L[lout].d, l.pk_fwd, l.Kf, l.Nf,
                               o, s);
    };
    int e = 0;
    const int c1 = kChan[0], c2 = kChan[1], c3 = kChan[2], c4 = kChan[3];
    e |= conv(0, dn::G_CONV3, d->xin, kInPadded, nullptr, 0, 0, 0, S_ENC1A);
    e |= conv(1, dn::G_CONV3, d->act[S_ENC1A], c1, nullptr, 0, 0, 0, S_ENC1B);
    e |= conv(2, dn::G_DOWN, d->act[S_ENC1B], c1, nullptr, 0, 0, 1, S_DOWN2);
    e |= conv(3, dn::G_CONV3, d->act[S_DOWN2], c2, nullptr, 0, 1, 1, S_ENC2A);
    e |= conv(4, dn::G_CONV3, d->act[S_ENC2A], c2, nullptr, 0, 1, 1, S_ENC2B);
    e |= conv(5, dn::G_DOWN, d->act[S_ENC2B], c2, nullptr, 0, 1, 2, S_DOWN3);
    e |= conv(6, dn::G_CONV3, d->act[S_DOWN3], c3, nullptr, 0, 2, 2, S_ENC3A);
    e |= conv(7, dn::G_CONV3, d->act[S_ENC3A], c3, nullptr, 0, 2, 2, S_ENC3B);
    e |= conv(8, dn::G_DOWN, d->act[S_ENC3B], c3, nullptr, 0, 2, 3, S_DOWN4);
    e |= conv(9, dn::G_CONV3, d->act[S_DOWN4], c4, nullptr, 0, 3, 3, S_ENC4A);
    e |= conv(10, dn::G_CONV3, d->act[S_ENC4A], c4, nullptr, 0, 3, 3, S_ENC4B);
    e |= conv(11, dn::G_UP, d->act[S_ENC4B], c4, nullptr, 0, 3, 2, S_UP3);
    e |= conv(12, dn::G_CONV3, d->act[S_ENC3B], c3, d->act[S_UP3], c3, 2, 2, S_DEC3A);
    e |= conv(13, dn::G_CONV3, d->act[S_DEC3A], c3, nullptr, 0, 2, 2, S_DEC3B);
    e |= conv(14, dn::G_UP, d->act[S_DEC3B], c3, nullptr, 0, 2, 1, S_UP2);
    e |= conv(15, dn::G_CONV3, d->act[S_ENC2B], c2, d->act[S_UP2], c2, 1, 1, S_DEC2A);
    e |= conv(16, dn::G_CONV3, d->act[S_DEC2A], c2, nullptr, 0, 1, 1, S_DEC2B);
    e |= conv(17, dn::G_UP, d->act[S_DEC2B], c2, nullptr, 0, 1, 0, S_UP1);
    e |= conv(18, dn::G_CONV3, d->act[S_ENC1B], c1, d->act[S_UP1], c1, 0, 0, S_DEC1A);
    e |= conv(19, dn::G_CONV3, d->act[S_DEC1A], c1, nullptr, 0, 0, 0, S_DEC1B);
    if (e) return dn_fail(d, OMC_EDEVICE, "convolution launch failed");
    const Layer& h = layer(d, 20);
    if (dn::launch_head_fwd(d->act[S_DEC1B], d->p + h.w_off, d->p + h.b_off, dose, inv_dmax, n,
                            d->y, out, s))
        return dn_fail(d, OMC_EDEVICE, "head launch failed");
    return OMC_OK;
}

// loss and gradient of every parameter into d->gp (after forward_pass)
int backward_pass(omc_dn* d, const float* target, float inv_dmax, hipStream_t s)
{
    const Level* L = d->lv;
    const size_t n = L[0].n;
    if (omc::launch_zero(d->gp, (d->n_params + 1) / 2, s) || omc::launch_zero(d->sums, 2, s))
        return dn_fail(d, OMC_EDEVICE, "zero-fill launch failed");
    if (dn::launch_loss(d->y, target, inv_dmax, n, d->sums, d->gy, s))
        return dn_fail(d, OMC_EDEVICE, "loss launch failed");
    const Layer& h = layer(d, 20);
    if (dn::launch_head_bwd(d->act[S_DEC1B], d->gy, d->p + h.w_off, n, d->gp + h.w_off,
                            d->gp + h.b_off, d->grad[S_DEC1B], s))
        return dn_fail(d, OMC_EDEVICE, "head backward launch failed");

    int e = 0;
    // masked gradient of layer li's output (slot, level lv, c channels) into scratch
    auto mask = [&](int slot, int lv, int c) {
        return dn::launch_relu_bwd(d->grad[slot], d->act[slot], L[lv].n * size_t(c), d->scratch, s);
    };
    auto wgrad = [&](int li, int geometry, const uint16_t* x0, int c0, const uint16_t* x1, int c1,
                     int lin, int lout) {
        const Layer& l = layer(d, li);
        return dn::launch_conv_wgrad(geometry, x0, c0, x1, c1, L[lin].d, L[lout].d, d->scratch,
                                     l.cout, l.cin_log, d->gp + l.w_off, d->gp + l.b_off, s);
    };
    // input gradient: conv over the masked output gradient with the backward packing
    auto dgrad = [&](int li, int geometry, int lrow_in, int lrow_out, float* g0, int split,
                     float* g1, int acc0) {
        const Layer& l = layer(d, li);
        dn::ConvOut o;
        o.g0 = g0;
        o.g1 = g1;
        o.split = split;
        o.acc0 = acc0;
        return dn::launch_conv(geometry, d->scratch, l.cout, nullptr, 0, L[lrow_in].d,
                               L[lrow_out].d, l.pk_bwd, l.Kb, l.Nb, o, s);
    };
    const int C[4] = {kChan[0], kChan[1], kChan[2], kChan[3]};
    // decoder, full resolution first
    const int decb[3] = {19, 16, 13}, deca[3] = {18, 15, 12}, upl[3] = {17, 14, 11};
    const int s_decb[3] = {S_DEC1B, S_DEC2B, S_DEC3B}, s_deca[3] = {S_DEC1A, S_DEC2A, S_DEC3A};
    const int s_up[3] = {S_UP1, S_UP2, S_UP3}, s_encb[4] = {S_ENC1B, S_ENC2B, S_ENC3B, S_ENC4B};
    const int s_enca[4] = {S_ENC1A, S_ENC2A, S_ENC3A, S_ENC4A};
    const int s_down[4] = {-1, S_DOWN2, S_DOWN3, S_DOWN4};
    for (int i = 0; i < 3; ++i) {
        const int c = C[i];
        e |= mask(s_decb[i], i, c);
        e |= wgrad(decb[i], dn::G_CONV3, d->act[s_deca[i]], c, nullptr, 0, i, i);
        e |= dgrad(decb[i], dn::G_CONV3, i, i, d->grad[s_deca[i]], c, nullptr, 0);
        e |= mask(s_deca[i], i, c);
        e |= wgrad(deca[i], dn::G_CONV3, d->act[s_encb[i]], c, d->act[s_up[i]], c, i, i);
        e |= dgrad(deca[i], dn::G_CONV3, i, i, d->grad[s_encb[i]], c, d->grad[s_up[i]], 0);
        e |= mask(s_up[i], i, c);
        const int s_prev = i == 2 ? S_ENC4B : s_decb[i + 1];
        e |= wgrad(upl[i], dn::G_UP, d->act[s_prev], C[i + 1], nullptr, 0, i + 1, i);
        // input gradient of the up layer: a 2x2x2 stride-2 window over its output gradient
        e |= dgrad(upl[i], dn::G_DOWN, i, i + 1, d->grad[s_prev], C[i + 1], nullptr, 0);
    }
    // encoder, coarsest first
    const int encb[4] = {1, 4, 7, 10}, enca[4] = {0, 3, 6, 9}, downl[4] = {-1, 2, 5, 8};
    for (int i = 3; i >= 0; --i) {
        const int c = C[i];
        e |= mask(s_encb[i], i, c);
        e |= wgrad(encb[i], dn::G_CONV3, d->act[s_enca[i]], c, nullptr, 0, i, i);
        e |= dgrad(encb[i], dn::G_CONV3, i, i, d->grad[s_enca[i]], c, nullptr, 0);
        e |= mask(s_enca[i], i, c);
        if (i == 0) {
            e |= wgrad(enca[0], dn::G_CONV3, d->xin, kInPadded, nullptr, 0, 0, 0);
            break;
        }
        e |= wgrad(enca[i], dn::G_CONV3, d->act[s_down[i]], c, nullptr, 0, i, i);
        e |= dgrad(enca[i], dn::G_CONV3, i, i, d->grad[s_down[i]], c, nullptr, 0);
        e |= mask(s_down[i], i, c);
        e |= wgrad(downl[i], dn::G_DOWN, d->act[s_encb[i - 1]], C[i - 1], nullptr, 0, i - 1, i);
        // input gradient of the down layer: a transposed 2x2x2 scatter, added to
        // the skip gradient the decoder left in the same buffer
        e |= dgrad(downl[i], dn::G_UP, i, i - 1, d->grad[s_encb[i - 1]], C[i - 1], nullptr, 1);
    }
    if (e) return dn_fail(d, OMC_EDEVICE, "backward launch failed");
    return OMC_OK;
}

int read_loss(omc_dn* d, hipStream_t s, float* loss)
{
    if (hipMemcpyAsync(d->h_sums, d->sums, 4 * sizeof(float), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return dn_fail(d, OMC_EDEVICE, "loss readback failed");
    if (loss) *loss = d->h_sums[1] > 0 ? d->h_sums[2] / d->h_sums[1] : 0.f;
    if (!std::isfinite(d->h_sums[2])) return dn_fail(d, OMC_ENUMERIC, "non-finite loss");
    return OMC_OK;
}

bool dmax_ok(double dmax) { return std::isfinite(dmax) && dmax > 0; }

__global__ void __launch_bounds__(256)
sigma_kernel(const double* __restrict__ dose, const double* __restrict__ dose2, int B, size_t n,
             float* __restrict__ d32, float* __restrict__ s32)
{
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double d = dose[v];
    const double var = B > 1 ? (dose2[v] / B - d * d) / (B - 1) : 0.0;
    d32[v] = float(d);
    s32[v] = float(var > 0 ? sqrt(var) : 0.0);
}

__global__ void __launch_bounds__(256)
combine_kernel(const double* __restrict__ a, double wa, const double* __restrict__ b, double wb,
               size_t n, float* __restrict__ out)
{
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < n) out[v] = float(wa * a[v] + wb * b[v]);
}

}  // namespace

extern "C" {

int omc_dn_create(omc_dn** out, int nx, int ny, int nz, uint32_t seed)
{
    if (!out) return dn_fail(nullptr, OMC_EINVAL, "out is NULL");
    *out = nullptr;
    const int dims[3] = {nx, ny, nz};
    for (int k : dims)
        if (k < 8 || k > 512 || k % 8)
            return dn_fail(nullptr, OMC_EINVAL, "volume sides must be multiples of 8 in 8..512");
    omc_dn* d = new (std::nothrow) omc_dn();
    if (!d) return dn_fail(nullptr, OMC_ENOMEM, "host allocation failed");
    if (hipGetDevice(&d->device) != hipSuccess) {
        delete d;
        return dn_fail(nullptr, OMC_EDEVICE, "no HIP device available");
    }
    for (int l = 0; l < kLevels; ++l) {
        d->lv[l].d = dn::Dims{nz >> l, ny >> l, nx >> l};
        d->lv[l].n = d->lv[l].d.vox();
    }
    build_layers(d);
    bool ok = dalloc(d, d->p, d->n_params + 1) && dalloc(d, d->gp, d->n_params + 1) &&
              dalloc(d, d->m, d->n_params + 1) && dalloc(d, d->v, d->n_params + 1);
    for (Layer& l : d->layers) {
        if (l.kind == K_HEAD) continue;
        ok = ok && dalloc(d, l.pk_fwd, dn::pack_elems(l.Kf, l.Nf));
        if (l.need_bwd) ok = ok && dalloc(d, l.pk_bwd, dn::pack_elems(l.Kb, l.Nb));
    }
    // activation slot -> (level, channels)
    const int lvl[S_COUNT] = {0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0};
    const int ch[S_COUNT] = {16, 16, 32, 32, 32, 48, 48, 48, 64, 64, 64,
                             48, 48, 48, 32, 32, 32, 16, 16, 16};
    for (int sl = 0; sl < S_COUNT; ++sl) {
        const size_t e = d->lv[lvl[sl]].n * size_t(ch[sl]);
        ok = ok && dalloc(d, d->act[sl], e) && dalloc(d, d->grad[sl], e);
    }
    const size_t n = d->lv[0].n;
    ok = ok && dalloc(d, d->xin, n * kInPadded) && dalloc(d, d->scratch, n * 16) &&
         dalloc(d, d->y, n) && dalloc(d, d->gy, n) && dalloc(d, d->sums, 4) &&
         hipHostMalloc(&d->h_sums, 4 * sizeof(float)) == hipSuccess &&
         hipHostMalloc(&d->h_acc, 8 * sizeof(double)) == hipSuccess && dalloc(d, d->acc, 8);
    if (!ok) {
        omc_dn_destroy(d);
        return dn_fail(nullptr, OMC_ENOMEM, "device allocation failed");
    }
    // initial parameters on the host
    std::vector<float> h(d->n_params, 0.f);
    uint64_t idx = 0;
    for (const Layer& l : d->layers) {
        const double sd = std::sqrt(2.0 / double(l.taps * l.cin_log));
        const size_t nw = size_t(l.taps) * l.cin_log * l.cout;
        for (size_t i = 0; i < nw; ++i) h[l.w_off + i] = float(sd * normal_of(seed, idx++));
    }
    const int rc = omc_dn_set_params(d, h.data(), d->n_params);
    if (rc) {
        omc_dn_destroy(d);
        return rc;
    }
    *out = d;
    return OMC_OK;
}

int omc_dn_num_params(const omc_dn* d, uint64_t* n)
{
    if (!d || !n) return dn_fail(nullptr, OMC_EINVAL, "NULL argument");
    *n = d->n_params;
    return OMC_OK;
}

int omc_dn_get_params(omc_dn* d, float* params, uint64_t n)
{
    if (!d || !params || n != d->n_params) return dn_fail(d, OMC_EINVAL, "need n == num_params");
    if (hipSetDevice(d->device) != hipSuccess ||
        hipMemcpy(params, d->p, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return dn_fail(d, OMC_EDEVICE, "parameter readback failed");
    return OMC_OK;
}

int omc_dn_set_params(omc_dn* d, const float* params, uint64_t n)
{
    if (!d || !params || n != d->n_params) return dn_fail(d, OMC_EINVAL, "need n == num_params");
    for (uint64_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return dn_fail(d, OMC_EINVAL, "non-finite parameter");
    if (hipSetDevice(d->device) != hipSuccess ||
        hipMemcpy(d->p, params, n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(d->m, 0, n * sizeof(float)) != hipSuccess ||
        hipMemset(d->v, 0, n * sizeof(float)) != hipSuccess)
        return dn_fail(d, OMC_EDEVICE, "parameter upload failed");
    d->step = 0;
    const int rc = repack(d, nullptr);
    if (rc) return rc;
    if (hipDeviceSynchronize() != hipSuccess) return dn_fail(d, OMC_EDEVICE, "weight packing failed");
    return OMC_OK;
}

int omc_dn_forward(omc_dn* d, const float* dose, const float* sigma, const float* rho, double dmax,
                   float* out, void* hip_stream)
{
    if (!d || !dose || !sigma || !rho || !out) return dn_fail(d, OMC_EINVAL, "NULL argument");
    if (!dmax_ok(dmax)) return dn_fail(d, OMC_EINVAL, "dmax must be finite and > 0");
    if (hipSetDevice(d->device) != hipSuccess) return dn_fail(d, OMC_EDEVICE, "hipSetDevice failed");
    (void)hipGetLastError();
    return forward_pass(d, dose, sigma, rho, float(1.0 / dmax), out,
                        static_cast<hipStream_t>(hip_stream));
}

int omc_dn_gradient(omc_dn* d, const float* dose, const float* sigma, const float* rho,
                    double dmax, const float* target, float* grad, uint64_t n, float* loss,
                    void* hip_stream)
{
    if (!d || !dose || !sigma || !rho || !target || !grad)
        return dn_fail(d, OMC_EINVAL, "NULL argument");
    if (n != d->n_params) return dn_fail(d, OMC_EINVAL, "need n == num_params");
    if (!dmax_ok(dmax)) return dn_fail(d, OMC_EINVAL, "dmax must be finite and > 0");
    if (hipSetDevice(d->device) != hipSuccess) return dn_fail(d, OMC_EDEVICE, "hipSetDevice failed");
    (void)hipGetLastError();
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const float inv = float(1.0 / dmax);
    int rc = forward_pass(d, dose, sigma, rho, inv, nullptr, s);
    if (!rc) rc = backward_pass(d, target, inv, s);
    if (!rc) rc = read_loss(d, s, loss);
    if (!rc && (hipMemcpyAsync(grad, d->gp, n * sizeof(float), hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess))
        rc = dn_fail(d, OMC_EDEVICE, "gradient readback failed");
    return rc;
}

int omc_dn_train_step(omc_dn* d, const float* dose, const float* sigma, const float* rho,
                      double dmax, const float* target, double lr, float* loss, void* hip_stream)
{
    if (!d || !dose || !sigma || !rho || !target) return dn_fail(d, OMC_EINVAL, "NULL argument");
    if (!dmax_ok(dmax) || !(lr > 0) || !std::isfinite(lr))
        return dn_fail(d, OMC_EINVAL, "dmax and lr must be finite and > 0");
    if (hipSetDevice(d->device) != hipSuccess) return dn_fail(d, OMC_EDEVICE, "hipSetDevice failed");
    (void)hipGetLastError();
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const float inv = float(1.0 / dmax);
    int rc = forward_pass(d, dose, sigma, rho, inv, nullptr, s);
    if (!rc) rc = backward_pass(d, target, inv, s);
    if (rc) return rc;
    d->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = float(1.0 - std::pow(b1, d->step));
    const float bc2 = float(1.0 - std::pow(b2, d->step));
    if (dn::launch_adam(d->p, d->m, d->v, d->gp, d->n_params, float(lr), float(b1), float(b2),
                        1e-8f, bc1, bc2, s))
        return dn_fail(d, OMC_EDEVICE, "Adam launch failed");
    if ((rc = repack(d, s))) return rc;
    return read_loss(d, s, loss);
}

namespace {
// True when [p, p + bytes) lies inside one HIP allocation of the network's
// device, so that a caller's buffer is checked before any kernel touches it.
bool on_device(const omc_dn* d, const void* p, size_t bytes)
{
    hipPointerAttribute_t at{};
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    const bool dev = hipPointerGetAttributes(&at, p) == hipSuccess &&
                     at.type == hipMemoryTypeDevice && at.device == d->device;
    const bool range =
        dev && hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess &&
        reinterpret_cast<uintptr_t>(p) >= reinterpret_cast<uintptr_t>(base) &&
        reinterpret_cast<uintptr_t>(p) + bytes <= reinterpret_cast<uintptr_t>(base) + size;
    (void)hipGetLastError();
    return dev && range && reinterpret_cast<uintptr_t>(p) % alignof(float) == 0;
}
}  // namespace

int omc_dn_denoise(omc_dn* d, omc_ctx* ctx, uint64_t n_low, uint32_t seed, uint32_t h0,
                   const float* d_rho, double max_err, uint64_t n_fallback, float* out,
                   double* err, int* fell_back, void* hip_stream)
{
    if (!d || !ctx || !d_rho || !out || !err || !fell_back)
        return dn_fail(d, OMC_EINVAL, "NULL argument");
    if (n_low == 0 || !(max_err >= 0)) return dn_fail(d, OMC_EINVAL, "need n_low >= 1, max_err >= 0");
    if (hipSetDevice(d->device) != hipSuccess) return dn_fail(d, OMC_EDEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t n = d->lv[0].n;
    // the engine writes its dose grids into buffers sized for the network's
    // volume: the phantom must have exactly the network's dimensions
    int nx = 0, ny = 0, nz = 0;
    if (omc_get_geometry(ctx, &nx, &ny, &nz, nullptr, nullptr, nullptr) != OMC_OK)
        return dn_fail(d, OMC_EINVAL, "invalid context");
    if (nx != d->lv[0].d.nx || ny != d->lv[0].d.ny || nz != d->lv[0].d.nz)
        return dn_fail(d, OMC_EINVAL, "the context's phantom (" + std::to_string(nx) + " x " +
                                          std::to_string(ny) + " x " + std::to_string(nz) +
                                          ") does not have the network's dimensions (" +
                                          std::to_string(d->lv[0].d.nx) + " x " +
                                          std::to_string(d->lv[0].d.ny) + " x " +
                                          std::to_string(d->lv[0].d.nz) + ")");
    if (!on_device(d, d_rho, n * sizeof(float)) || !on_device(d, out, n * sizeof(float)))
        return dn_fail(d, OMC_EINVAL, "d_rho and out must be allocations of the network's "
                                      "device holding one float per voxel");
    if (!d->d64 && !(dalloc(d, d->d64, 4 * n) && dalloc(d, d->f32, 2 * n)))
        return dn_fail(d, OMC_ENOMEM, "device allocation failed");
    omc_params prm;
    if (omc_get_params(ctx, &prm) != OMC_OK) return dn_fail(d, OMC_EINVAL, "invalid context");
    int rc = omc_run_device(ctx, n_low, seed, h0, d->d64, d->d64 + n, hip_stream);
    if (rc != OMC_OK) return dn_fail(d, rc, std::string("Monte Carlo run failed: ") + omc_last_error(ctx));
    const unsigned grid = unsigned((n + 255) / 256);
    float* lo = d->f32;
    float* sg = d->f32 + n;
    hipLaunchKernelGGL(sigma_kernel, dim3(grid), dim3(256), 0, s, d->d64, d->d64 + n,
                       prm.n_batches, n, lo, sg);
    if (omc::launch_zero(d->acc, 8, s) || hipGetLastError() != hipSuccess)
        return dn_fail(d, OMC_EDEVICE, "launch failed");
    // maximum of the low-history dose for the normalisation
    if (dn::launch_dn_error(lo, lo, sg, n, d->acc, s) ||
        hipMemcpyAsync(d->h_acc, d->acc, 8 * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return dn_fail(d, OMC_EDEVICE, "normalisation failed");
    const double dmax = d->h_acc[0];
    if (!dmax_ok(dmax)) return dn_fail(d, OMC_ENUMERIC, "the low-history dose is empty");
    if ((rc = forward_pass(d, lo, sg, d_rho, float(1.0 / dmax), out, s))) return rc;
    if (omc::launch_zero(d->acc, 8, s) || dn::launch_dn_error(out, lo, sg, n, d->acc, s) ||
        hipMemcpyAsync(d->h_acc, d->acc, 8 * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return dn_fail(d, OMC_EDEVICE, "error estimate failed");
    const double cnt = std::max(d->h_acc[1], 1.0);
    const double excess = d->h_acc[2] / cnt - d->h_acc[3] / cnt;
    *err = std::sqrt(std::max(excess, 0.0)) / dmax;
    *fell_back = 0;
    if (*err > max_err && n_fallback > 0) {
        if (uint64_t(h0) + n_low + n_fallback > (uint64_t(1) << 32))
            return dn_fail(d, OMC_EINVAL, "history range of the fallback exceeds 2^32");
        rc = omc_run_device(ctx, n_fallback, seed, uint32_t(h0 + n_low), d->d64 + 2 * n,
                            d->d64 + 3 * n, hip_stream);
        if (rc != OMC_OK)
            return dn_fail(d, rc, std::string("fallback run failed: ") + omc_last_error(ctx));
        const double tot = double(n_low + n_fallback);
        hipLaunchKernelGGL(combine_kernel, dim3(grid), dim3(256), 0, s, d->d64, double(n_low) / tot,
                           d->d64 + 2 * n, double(n_fallback) / tot, n, out);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return dn_fail(d, OMC_EDEVICE, "combine launch failed");
        *fell_back = 1;
    }
    return OMC_OK;
}

int omc_dn_debug_layer(int geometry, int nx, int ny, int nz, int c0, int c1, int cout,
                       const float* x, const float* w, const float* b, const float* gy,
                       float* y, float* gx, float* gw, float* gb)
{
    if (!x || !w || geometry < 0 || geometry > 2 || c0 < 8 || c0 % 8 || c1 < 0 || c1 % 8 ||
        cout < 16 || cout % 16 || nx < 1 || ny < 1 || nz < 1 || nx > 256 || ny > 256 ||
        nz > 256 || (geometry == dn::G_DOWN && (nx % 2 || ny % 2 || nz % 2)))
        return dn_fail(nullptr, OMC_EINVAL, "invalid layer test arguments");
    if ((gx || gw || gb) && !gy) return dn_fail(nullptr, OMC_EINVAL, "gradients need gy");
    if (gx && (c0 + c1) % 16) return dn_fail(nullptr, OMC_EINVAL, "gx needs c0 + c1 % 16 == 0");
    const int cin = c0 + c1;
    const int taps = geometry == dn::G_CONV3 ? 27 : 8;
    const dn::Dims in{nz, ny, nx};
    const dn::Dims out = geometry == dn::G_CONV3 ? in
                         : geometry == dn::G_DOWN ? dn::Dims{nz / 2, ny / 2, nx / 2}
                                                  : dn::Dims{2 * nz, 2 * ny, 2 * nx};
    const size_t ni = in.vox(), no = out.vox();
    const size_t nw = size_t(taps) * cin * cout;
    omc_dn tmp;  // only its allocation list and error string are used
    auto bail = [&](int code, const char* msg) {
        for (void* q : tmp.allocs) (void)hipFree(q);
        return dn_fail(nullptr, code, msg);
    };
    float *dx32 = nullptr, *dw = nullptr, *db = nullptr, *dgy32 = nullptr, *dgx = nullptr,
          *dgw = nullptr, *dgb = nullptr, *dy = nullptr;
    uint16_t *dx0 = nullptr, *dx1 = nullptr, *dgy = nullptr, *pk = nullptr, *ybf = nullptr;
    const int Kf = geometry == dn::G_UP ? cin : taps * cin;
    const int Nf = geometry == dn::G_UP ? 8 * cout : cout;
    const int Kb = geometry == dn::G_DOWN ? cout : taps * cout;
    const int Nb = geometry == dn::G_DOWN ? 8 * cin : cin;
    bool ok = dalloc(&tmp, dx32, ni * cin) && dalloc(&tmp, dw, nw) && dalloc(&tmp, db, cout) &&
              dalloc(&tmp, dgy32, no * cout) && dalloc(&tmp, dgx, ni * cin) &&
              dalloc(&tmp, dgw, nw) && dalloc(&tmp, dgb, cout) && dalloc(&tmp, dy, no * cout) &&
              dalloc(&tmp, dx0, ni * c0) && dalloc(&tmp, dx1, ni * std::max(c1, 8)) &&
              dalloc(&tmp, dgy, no * cout) && dalloc(&tmp, ybf, no * cout) &&
              dalloc(&tmp, pk, std::max(dn::pack_elems(Kf, Nf), dn::pack_elems(Kb, Nb)));
    if (!ok) return bail(OMC_ENOMEM, "device allocation failed");
    // split x into its two sources (BF16), weights and gradients
    std::vector<float> h0(ni * c0), h1(ni * std::max(c1, 1));
    for (size_t v = 0; v < ni; ++v) {
        for (int c = 0; c < c0; ++c) h0[v * c0 + c] = x[v * cin + c];
        for (int c = 0; c < c1; ++c) h1[v * c1 + c] = x[v * cin + c0 + c];
    }
    std::vector<float> hb(cout, 0.f);
    if (b) hb.assign(b, b + cout);
    int e = 0;
    e |= hipMemcpy(dx32, h0.data(), ni * c0 * sizeof(float), hipMemcpyHostToDevice) != hipSuccess;
    e |= dn::launch_f32_to_bf16(dx32, ni * c0, dx0, nullptr);
    if (c1) {
        e |= hipDeviceSynchronize() != hipSuccess;
        e |= hipMemcpy(dx32, h1.data(), ni * c1 * sizeof(float), hipMemcpyHostToDevice) != hipSuccess;
        e |= dn::launch_f32_to_bf16(dx32, ni * c1, dx1, nullptr);
    }
    e |= hipMemcpy(dw, w, nw * sizeof(float), hipMemcpyHostToDevice) != hipSuccess;
    e |= hipMemcpy(db, hb.data(), cout * sizeof(float), hipMemcpyHostToDevice) != hipSuccess;
    if (gy) {
        e |= hipMemcpy(dgy32, gy, no * cout * sizeof(float), hipMemcpyHostToDevice) != hipSuccess;
        e |= dn::launch_f32_to_bf16(dgy32, no * cout, dgy, nullptr);
    }
    if (e || hipDeviceSynchronize() != hipSuccess) return bail(OMC_EDEVICE, "upload failed");
    if (y) {
        // forward with an FP32 result: run the input-gradient epilogue (FP32
        // columns) on the forward packing, then add the bias on the host side
        e |= dn::launch_pack(dw, taps, cin, cin, cout,
                             geometry == dn::G_UP ? dn::PACK_FWD_UP : dn::PACK_FWD, pk, nullptr);
        dn::ConvOut o;
        o.g0 = dy;
        o.split = cout;
        e |= dn::launch_conv(geometry, dx0, c0, c1 ? dx1 : nullptr, c1, in, out, pk, Kf, Nf, o,
                             nullptr);
        e |= hipDeviceSynchronize() != hipSuccess;
        e |= hipMemcpy(y, dy, no * cout * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess;
        for (size_t v = 0; v < no && !e; ++v)
            for (int c = 0; c < cout; ++c) y[v * cout + c] += hb[c];
    }
    if (gx && !e) {
        const int bm = geometry == dn::G_CONV3 ? dn::PACK_BWD_FLIP
                       : geometry == dn::G_UP  ? dn::PACK_BWD
                                               : dn::PACK_BWD_UP;
        e |= dn::launch_pack(dw, taps, cin, cin, cout, bm, pk, nullptr);
        dn::ConvOut o;
        o.g0 = dgx;
        o.split = cin;
        const int g_bwd = geometry == dn::G_CONV3 ? dn::G_CONV3
                          : geometry == dn::G_UP  ? dn::G_DOWN
                                                  : dn::G_UP;
        e |= dn::launch_conv(g_bwd, dgy, cout, nullptr, 0, out, in, pk, Kb, Nb, o, nullptr);
        e |= hipDeviceSynchronize() != hipSuccess;
        e |= hipMemcpy(gx, dgx, ni * cin * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess;
    }
    if ((gw || gb) && !e) {
        e |= hipMemset(dgw, 0, nw * sizeof(float)) != hipSuccess;
        e |= hipMemset(dgb, 0, cout * sizeof(float)) != hipSuccess;
        e |= dn::launch_conv_wgrad(geometry, dx0, c0, c1 ? dx1 : nullptr, c1, in, out, dgy, cout,
                                   cin, dgw, dgb, nullptr);
        e |= hipDeviceSynchronize() != hipSuccess;
        if (gw) e |= hipMemcpy(gw, dgw, nw * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess;
        if (gb) e |= hipMemcpy(gb, dgb, cout * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess;
    }
    for (void* q : tmp.allocs) (void)hipFree(q);
    tmp.allocs.clear();
    if (e) return dn_fail(nullptr, OMC_EDEVICE, "layer kernels failed");
    return OMC_OK;
}

const char* omc_dn_last_error(const omc_dn* d)
{
    if (d) return d->err.c_str();
    return g_dn_error.c_str();
}

void omc_dn_destroy(omc_dn* d)
{
    if (!d) return;
    for (void* q : d->allocs) (void)hipFree(q);
    if (d->h_sums) (void)hipHostFree(d->h_sums);
    if (d->h_acc) (void)hipHostFree(d->h_acc);
    delete d;
}

}  // extern "C"
