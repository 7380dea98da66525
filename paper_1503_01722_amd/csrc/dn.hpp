// dn.hpp -- learned dose denoiser: launchers of the gfx950 kernels.
//
// Tensors are channels-last: a volume of nz x ny x nx voxels with C channels
// is [voxel][C], voxel = x + nx (y + ny z). Activations and the operands of the
// matrix cores are BF16 (raw 16-bit patterns in memory), accumulation is FP32,
// master weights, optimiser state and activation gradients are FP32.
//
// Every convolution runs as an implicit GEMM on v_mfma_f32_16x16x32_bf16:
// rows are voxels, columns output channels, the reduction runs over (tap,
// input channel). Weights are stored pre-packed in the B-operand lane layout:
// packed[n_tile][k_block][lane][8], k_block of 32 reduction indices, n_tile of
// 16 columns, so that each lane loads its 8 BF16 with one 16-byte load.
#pragma once

#include <cstddef>
#include <cstdint>

namespace dn {

enum Geometry : int {
    G_CONV3 = 0,  // 3x3x3, stride 1, zero padding 1: out[v] reads in[v + t - 1]
    G_DOWN = 1,   // 2x2x2, stride 2: out[v] reads in[2 v + t]
    G_UP = 2      // 2x2x2 transposed, stride 2: out[2 v + t] reads in[v]
};

struct Dims {
    int nz, ny, nx;
    size_t vox() const { return size_t(nz) * ny * nx; }
};

// Packing of a logical FP32 weight W[t][ci][co] (ci < cin_log, zero for
// cin_log <= ci < cin) into the B layout of one GEMM view:
//   PACK_FWD      k = t * cin + ci, n = co             (conv3, down)
//   PACK_FWD_UP   k = ci,           n = t * cout + co  (up)
//   PACK_BWD_FLIP k = t * cout + co, n = ci, tap 26-t  (input gradient of conv3)
//   PACK_BWD      k = t * cout + co, n = ci            (input gradient of up)
//   PACK_BWD_UP   k = co,           n = t * cin + ci   (input gradient of down)
enum PackMode : int { PACK_FWD = 0, PACK_FWD_UP, PACK_BWD_FLIP, PACK_BWD, PACK_BWD_UP };

// Reduction blocks of 32 and column tiles of 16 of a GEMM view.
int pack_kblocks(int K);
int pack_ntiles(int N);
size_t pack_elems(int K, int N);

int launch_pack(const float* w, int taps, int cin_log, int cin, int cout, int mode,
                uint16_t* packed, void* stream);

// Forward / input-gradient convolution. Input: x0 (c0 channels) and, when c1 >
// 0, x1 (c1 channels) concatenated after it; both multiples of 8. geometry
// selects the gather (G_CONV3, G_DOWN: rows are output voxels of `out`; G_UP:
// rows are input voxels and columns (t, co) scatter to 2 v + t).
// K = taps * (c0 + c1) for the window geometries, c0 + c1 for G_UP; N = the
// packed columns (cout, or 8 * cout for G_UP).
// Epilogue: y (BF16, [vox_out][N_out]) with bias and optional ReLU, or FP32
// columns split at `split`: columns < split go to g0 ([vox][split]), the rest
// to g1 ([vox][N_out - split]); acc0/acc1 add to what is there.
struct ConvOut {
    uint16_t* y = nullptr;
    const float* bias = nullptr;
    int relu = 0;
    float* g0 = nullptr;
    float* g1 = nullptr;
    int split = 0;
    int acc0 = 0, acc1 = 0;
};
int launch_conv(int geometry, const uint16_t* x0, int c0, const uint16_t* x1, int c1, Dims in,
                Dims out, const uint16_t* packed, int K, int N, const ConvOut& o, void* stream);

// Weight (and bias) gradient: gw[t][ci][co] += sum over rows of A_t[row][ci]
// * G_t[row][co] for ci < cin_log, with A the (concatenated) input gathered as
// in the forward pass and G the masked output gradient (BF16, [vox_out][cout]).
// gb[co] += sum of G over the output voxels (may be NULL).
int launch_conv_wgrad(int geometry, const uint16_t* x0, int c0, const uint16_t* x1, int c1,
                      Dims in, Dims out, const uint16_t* g, int cout, int cin_log, float* gw,
                      float* gb, void* stream);

// Elementwise and reduction kernels.
int launch_pack_input(const float* dose, const float* sigma, const float* rho, float inv_dmax,
                      size_t n, uint16_t* x, void* stream);
// delta = dec . wh + bh; y = dose * inv_dmax + delta (normalised); out = y * dmax
int launch_head_fwd(const uint16_t* dec, const float* wh, const float* bh, const float* dose,
                    float inv_dmax, size_t n, float* y, float* out, void* stream);
// loss on normalised y and target t = target * inv_dmax: sums[0] = max t,
// sums[1] = sum w, sums[2] = sum w r^2 (all FP32 in device memory), then gy.
int launch_loss(const float* y, const float* target, float inv_dmax, size_t n, float* sums,
                float* gy, void* stream);
// gwh[c] += sum gy dec[:, c]; gbh += sum gy; gdec[v][c] = gy[v] wh[c]
int launch_head_bwd(const uint16_t* dec, const float* gy, const float* wh, size_t n, float* gwh,
                    float* gbh, float* gdec, void* stream);
// out = bf16(g * (act > 0))
int launch_relu_bwd(const float* g, const uint16_t* act, size_t n, uint16_t* out, void* stream);
int launch_adam(float* p, float* m, float* v, const float* g, size_t n, float lr, float b1,
                float b2, float eps, float bc1, float bc2, void* stream);
int launch_f32_to_bf16(const float* in, size_t n, uint16_t* out, void* stream);
int launch_bf16_to_f32(const uint16_t* in, size_t n, float* out, void* stream);
// error estimate of a denoised dose against the low-history run it came from:
// over voxels with lo > 0.1 max(lo): acc[0] = max lo, acc[1] = count,
// acc[2] = sum (dn - lo)^2, acc[3] = sum sigma^2 (FP64 sums)
int launch_dn_error(const float* dn, const float* lo, const float* sigma, size_t n, double* acc,
                    void* stream);

}  // namespace dn
