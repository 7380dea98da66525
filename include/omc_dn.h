/*
 * omc_dn.h -- C ABI of the learned dose denoiser that accompanies the Monte
 * Carlo engine of omc.h. The paper has no denoiser (its speed-ups come from
 * the GPU transport alone, Sec. 3); this network is the learned extension of
 * the method: a 3D U-Net maps a low-history dose, its batch uncertainty
 * (Sec. 3.1) and the density to the dose of a high-history run, with plain
 * Monte Carlo as the fallback and as the judge of its error.
 *
 * Network: level channels 16, 32, 48, 64; per level two 3x3x3 convolutions
 * (stride 1, zero padding 1) with ReLU; 2x2x2 stride-2 convolutions down and
 * 2x2x2 stride-2 transposed convolutions up (each with ReLU); the decoder
 * concatenates [skip, up]; a 1x1x1 head gives delta and the output is
 * D_low + delta * Dmax_low. Inputs are normalised as [D_low / Dmax_low,
 * sigma_low / Dmax_low, rho / 2]. Weights and activations are BF16 on the
 * matrix cores with FP32 accumulation; master weights, gradients and Adam
 * state are FP32.
 *
 * Parameter vector (float32): layer by layer in the order enc1a enc1b down2
 * enc2a enc2b down3 enc3a enc3b down4 enc4a enc4b up3 dec3a dec3b up2 dec2a
 * dec2b up1 dec1a dec1b head, each the weight [kz][ky][kx][c_in][c_out] then
 * the bias [c_out] (kernel 3 for enc/dec, 2 for down/up, 1 for head; c_in of
 * enc1a is 3, of dec{l}a twice the level's channels).
 *
 * Conventions as in omc.h: status return codes (OMC_OK / OMC_E*), host arrays
 * copied during the call, device pointers caller-owned and valid on the given
 * stream (NULL = default stream), one thread at a time per object. Volumes
 * are nz x ny x nx float32 arrays with x fastest; nx, ny, nz must be
 * multiples of 8 in 8..512.
 */
#ifndef OMC_DN_H
#define OMC_DN_H

#include <stdint.h>

#include "omc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct omc_dn omc_dn;

/* Create a network for volumes of nz x ny x nx voxels on the current device,
 * He-normal weights from a counter-based generator keyed by seed, zero biases,
 * Adam state zero. Allocates weights, optimiser state and every activation and
 * gradient buffer of one volume. */
int omc_dn_create(omc_dn** out, int nx, int ny, int nz, uint32_t seed);

/* Number of float32 parameters (the same for every volume size). */
int omc_dn_num_params(const omc_dn* dn, uint64_t* n);

/* Copy the FP32 master parameters to host memory (n = omc_dn_num_params). */
int omc_dn_get_params(omc_dn* dn, float* params, uint64_t n);

/* Replace the parameters from host memory; resets the Adam state and step. */
int omc_dn_set_params(omc_dn* dn, const float* params, uint64_t n);

/* Denoise: d_out = D_low + delta * dmax for device volumes d_dose (D_low),
 * d_sigma (its standard error) and d_rho (density), dmax > 0 the
 * normalisation (normally max D_low). */
int omc_dn_forward(omc_dn* dn, const float* d_dose, const float* d_sigma, const float* d_rho,
                   double dmax, float* d_out, void* hip_stream);

/* One training step on one volume: forward, weighted MSE against d_target
 * (same units as d_dose; weight 1 where target / dmax > 0.1 max, else 0.1),
 * backward through every layer, Adam update (lr, beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected). *loss receives the loss before the update. */
int omc_dn_train_step(omc_dn* dn, const float* d_dose, const float* d_sigma, const float* d_rho,
                      double dmax, const float* d_target, double lr, float* loss,
                      void* hip_stream);

/* Loss and its gradient with respect to every parameter (host memory, n
 * floats) for one volume, without an update (used to check the backward pass
 * against the reference implementation). */
int omc_dn_gradient(omc_dn* dn, const float* d_dose, const float* d_sigma, const float* d_rho,
                    double dmax, const float* d_target, float* grad, uint64_t n, float* loss,
                    void* hip_stream);

/* Denoised dose with plain Monte Carlo as fallback and judge: transports
 * n_low histories with ctx (its source and parameters; the phantom must have
 * the network's dimensions; d_rho is its density as a device float32 volume),
 * denoises the result, and estimates the error of
 * the denoised dose from the low-history run itself: over voxels with
 * D_low > 10 % of its maximum, err = sqrt(max(0, mean((D_dn - D_low)^2) -
 * mean(sigma_low^2))) / max D_low (the part of the difference its statistics
 * cannot explain). If err > max_err, n_fallback more histories (following
 * history ids) are transported and d_out is the plain Monte Carlo dose of all
 * n_low + n_fallback histories. d_out: device float32 volume. *err receives
 * the estimate, *fell_back 0 or 1. A phantom whose nx, ny, nz differ from the
 * network's, or d_rho / d_out that are not device allocations of the network's
 * device holding one float per voxel, give OMC_EINVAL before any launch. */
int omc_dn_denoise(omc_dn* dn, omc_ctx* ctx, uint64_t n_low, uint32_t seed, uint32_t h0,
                   const float* d_rho, double max_err, uint64_t n_fallback, float* d_out,
                   double* err, int* fell_back, void* hip_stream);

/* Test entry (host arrays in and out): one layer of the network's kinds on a
 * volume of nz x ny x nx input voxels. geometry 0: 3x3x3 stride 1 pad 1;
 * 1: 2x2x2 stride 2; 2: 2x2x2 transposed stride 2. x: [vox_in][c0 + c1]
 * (values rounded to BF16 by the call), the first c0 channels from one
 * source and the rest from a second (c1 may be 0); w: [taps][c0 + c1][cout];
 * b: [cout]; gy: [vox_out][cout] output gradient. Outputs (float32, any may be
 * NULL): y [vox_out][cout] = conv + bias without activation; gx [vox_in][c0
 * + c1] input gradient; gw [taps][c0 + c1][cout] and gb [cout] weight and
 * bias gradients. c0, c1, cout: multiples of 8 (c0 + c1 and cout of 16 for
 * gx). */
int omc_dn_debug_layer(int geometry, int nx, int ny, int nz, int c0, int c1, int cout,
                       const float* x, const float* w, const float* b, const float* gy,
                       float* y, float* gx, float* gw, float* gb);

const char* omc_dn_last_error(const omc_dn* dn);
void omc_dn_destroy(omc_dn* dn);

#ifdef __cplusplus
}
#endif
#endif
