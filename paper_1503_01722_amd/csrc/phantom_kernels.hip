// phantom_kernels.hip -- the phantom in device memory: the interleaved voxel
// records of the transport built from the plain density and material arrays,
// and the CT mapping (Sec. 2.1: each voxel's density and material from the
// patient's CT by a mapping method, after Schneider et al. 2000).
//
// Built with -ffp-contract=off: the interpolation below is FP64 with one
// rounding per operation, in a fixed order, so that the FP32 density it
// produces is the same bit pattern on any IEEE FP64 machine.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "engine.hpp"

namespace omc {

namespace {
inline int status() { return hipGetLastError() == hipSuccess ? 0 : -1; }
}  // namespace

// vox[v] = {density bits, slot of the voxel's material}: one 8-byte load per
// voxel visit in the transport kernels
__global__ void __launch_bounds__(256)
build_vox_kernel(const float* __restrict__ rho, const uint8_t* __restrict__ mat, size_t nvox,
                 const uint32_t* __restrict__ slot, uint2* __restrict__ vox)
{
    for (size_t v = size_t(blockIdx.x) * 256 + threadIdx.x; v < nvox;
         v += size_t(gridDim.x) * 256)
        vox[v] = make_uint2(__float_as_uint(rho[v]), slot[mat[v]]);
}

int launch_build_vox(const float* rho, const uint8_t* mat, size_t nvox, const uint32_t* slot,
                     uint32_t* vox, void* stream)
{
    const size_t blocks = std::min<size_t>((nvox + 255) / 256, 65536);
    hipLaunchKernelGGL(build_vox_kernel, dim3(unsigned(blocks)), dim3(256), 0,
                       (hipStream_t)stream, rho, mat, nvox, slot, reinterpret_cast<uint2*>(vox));
    return status();
}

// One voxel per work-item (grid-stride). map = [hu nodes][rho nodes][bin upper
// bounds] (FP64), bin_mat = material of each bin. Density: the end node's
// value outside the nodes, else rho_k + (h - hu_k) * ((rho_k+1 - rho_k) /
// (hu_k+1 - hu_k)) on the segment hu_k <= h < hu_k+1, rounded once to FP32.
// Material: the first bin with h < upper_b, else the last. rmax_bits[m] ends
// as the largest FP32 density bits of material m (positive floats order as
// their bit patterns), reduced per work-group in LDS first.
__global__ void __launch_bounds__(256)
ct_map_kernel(const int16_t* __restrict__ hu, size_t nvox, const double* __restrict__ map,
              const uint32_t* __restrict__ bin_mat, int n_nodes, int n_bins,
              float* __restrict__ rho, uint8_t* __restrict__ mat, uint32_t* __restrict__ rmax_bits)
{
    __shared__ double s_map[2 * kMaxCtNodes + kMaxCtBins];
    __shared__ uint32_t s_mat[kMaxCtBins];
    __shared__ uint32_t s_max[kMaxMaterials];
    const int n_map = 2 * n_nodes + n_bins;
    for (int k = threadIdx.x; k < n_map; k += 256) s_map[k] = map[k];
    for (int k = threadIdx.x; k < n_bins; k += 256) s_mat[k] = bin_mat[k];
    for (int k = threadIdx.x; k < kMaxMaterials; k += 256) s_max[k] = 0u;
    __syncthreads();
    const double* H = s_map;
    const double* P = s_map + n_nodes;
    const double* U = s_map + 2 * n_nodes;
    for (size_t v = size_t(blockIdx.x) * 256 + threadIdx.x; v < nvox;
         v += size_t(gridDim.x) * 256) {
        const double h = double(hu[v]);
        double r;
        if (h <= H[0]) {
            r = P[0];
        } else if (h >= H[n_nodes - 1]) {
            r = P[n_nodes - 1];
        } else {
            int k = 0;
            while (k + 2 < n_nodes && H[k + 1] <= h) ++k;
            const double slope = (P[k + 1] - P[k]) / (H[k + 1] - H[k]);
            r = P[k] + (h - H[k]) * slope;
        }
        int b = 0;
        while (b + 1 < n_bins && !(h < U[b])) ++b;
        const float rf = float(r);
        const uint32_t m = s_mat[b];
        rho[v] = rf;
        mat[v] = uint8_t(m);
        atomicMax(&s_max[m], __float_as_uint(rf));
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kMaxMaterials; k += 256)
        if (s_max[k]) atomicMax(&rmax_bits[k], s_max[k]);
}

int launch_ct_map(const int16_t* hu, size_t nvox, const double* map, const uint32_t* bin_mat,
                  int n_nodes, int n_bins, float* rho, uint8_t* mat, uint32_t* rmax_bits,
                  void* stream)
{
    const size_t blocks = std::min<size_t>((nvox + 255) / 256, 16384);
    hipLaunchKernelGGL(ct_map_kernel, dim3(unsigned(blocks)), dim3(256), 0, (hipStream_t)stream,
                       hu, nvox, map, bin_mat, n_nodes, n_bins, rho, mat, rmax_bits);
    return status();
}

}  // namespace omc
