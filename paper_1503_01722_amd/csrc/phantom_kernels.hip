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

__global__ void __launch_bounds__(256)
cell_scale_kernel(const uint2* __restrict__ vox, int nx, int ny, int nz, int shift, int cnx,
                  int cny, const double* __restrict__ r, uint32_t* __restrict__ q)
{
    const size_t nvox = size_t(nx) * size_t(ny) * size_t(nz);
    for (size_t v = size_t(blockIdx.x) * 256 + threadIdx.x; v < nvox;
         v += size_t(gridDim.x) * 256) {
        const uint2 rec = vox[v];
        double qd = ceil(255.0 * (double(__uint_as_float(rec.x)) * r[rec.y]));
        qd = qd < 1.0 ? 1.0 : (qd > 255.0 ? 255.0 : qd);
        const int x = int(v % size_t(nx));
        const int y = int((v / size_t(nx)) % size_t(ny));
        const int z = int(v / (size_t(nx) * size_t(ny)));
        const int c = (x >> shift) + cnx * ((y >> shift) + cny * (z >> shift));
        atomicMax(&q[c], uint32_t(qd));
    }
}

int launch_cell_scales(const uint32_t* vox, int nx, int ny, int nz, int shift, int cnx, int cny,
                       const double* r, uint32_t* q, void* stream)
{
    const size_t nvox = size_t(nx) * size_t(ny) * size_t(nz);
    const size_t blocks = std::min<size_t>((nvox + 255) / 256, 16384);
    hipLaunchKernelGGL(cell_scale_kernel, dim3(unsigned(blocks)), dim3(256), 0,
                       (hipStream_t)stream, reinterpret_cast<const uint2*>(vox), nx, ny, nz,
                       shift, cnx, cny, r, q);
    return status();
}

// The CT mapping, in two launches. ct_lut_kernel evaluates the mapping once
// for each of the 65536 int16 HU values: map = [hu nodes][rho nodes][bin upper
// bounds][segment slopes (rho_k+1 - rho_k) / (hu_k+1 - hu_k), divided on the
// host: the same correctly rounded FP64 quotient the definition takes] and
// bin_mat = the material of each bin. Density: the end node's value outside
// the nodes, else rho_k + (h - hu_k) * slope_k on the segment hu_k <= h <
// hu_k+1, rounded once to FP32. Material: the first bin with h < upper_b, else
// the last. ct_map_kernel then maps every voxel by a lookup in that table
// (320 KB, L2-resident): one coalesced 2-byte read and 5 bytes written per
// voxel.
__global__ void __launch_bounds__(256)
ct_lut_kernel(const double* __restrict__ map, const uint32_t* __restrict__ bin_mat, int n_nodes,
              int n_bins, float* __restrict__ lut_rho, uint8_t* __restrict__ lut_mat)
{
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i >= kCtLutSize) return;
    const double* H = map;
    const double* P = map + n_nodes;
    const double* U = map + 2 * n_nodes;
    const double* S = map + 2 * n_nodes + n_bins;
    const double h = double(i - kCtLutSize / 2);
    double r;
    if (h <= H[0]) {
        r = P[0];
    } else if (h >= H[n_nodes - 1]) {
        r = P[n_nodes - 1];
    } else {
        int j = 0;
        while (j + 2 < n_nodes && H[j + 1] <= h) ++j;
        r = P[j] + (h - H[j]) * S[j];
    }
    int b = 0;
    while (b + 1 < n_bins && !(h < U[b])) ++b;
    lut_rho[i] = float(r);
    lut_mat[i] = uint8_t(bin_mat[b]);
}

// rmax_bits[m] ends as the largest FP32 density bits of material m (positive
// floats order as their bit patterns). Each work-item walks a column of
// kCtRun voxels 256 apart (coalesced across the work-group) and keeps the
// running maximum of its current material, so that the LDS maximum is taken
// when the material changes rather than once per voxel.
constexpr int kCtRun = 16;

__global__ void __launch_bounds__(256)
ct_map_kernel(const int16_t* __restrict__ hu, size_t nvox, const float* __restrict__ lut_rho,
              const uint8_t* __restrict__ lut_mat, float* __restrict__ rho,
              uint8_t* __restrict__ mat, uint32_t* __restrict__ rmax_bits)
{
    __shared__ uint32_t s_max[kMaxMaterials];
    for (int k = threadIdx.x; k < kMaxMaterials; k += 256) s_max[k] = 0u;
    __syncthreads();
    uint32_t cur_m = 0, cur_max = 0;
    auto one = [&](size_t v, int h) {
        const int i = h + kCtLutSize / 2;
        const float rf = lut_rho[i];
        const uint32_t m = lut_mat[i];
        rho[v] = rf;
        mat[v] = uint8_t(m);
        const uint32_t bits = __float_as_uint(rf);
        if (m == cur_m) {
            cur_max = bits > cur_max ? bits : cur_max;
        } else {
            if (cur_max) atomicMax(&s_max[cur_m], cur_max);
            cur_m = m;
            cur_max = bits;
        }
    };
    const size_t stride = size_t(gridDim.x) * 256 * kCtRun;
    for (size_t t0 = size_t(blockIdx.x) * 256 * kCtRun; t0 < nvox; t0 += stride) {
        if (t0 + size_t(256) * kCtRun <= nvox) {
            // a whole tile: all its HU loads in flight before the first lookup
            int hv[kCtRun];
#pragma unroll
            for (int k = 0; k < kCtRun; ++k) hv[k] = hu[t0 + size_t(k) * 256 + threadIdx.x];
#pragma unroll
            for (int k = 0; k < kCtRun; ++k) one(t0 + size_t(k) * 256 + threadIdx.x, hv[k]);
        } else {
            for (int k = 0; k < kCtRun; ++k) {
                const size_t v = t0 + size_t(k) * 256 + threadIdx.x;
                if (v >= nvox) break;
                one(v, hu[v]);
            }
        }
    }
    if (cur_max) atomicMax(&s_max[cur_m], cur_max);
    __syncthreads();
    for (int k = threadIdx.x; k < kMaxMaterials; k += 256)
        if (s_max[k]) atomicMax(&rmax_bits[k], s_max[k]);
}

int launch_ct_map(const int16_t* hu, size_t nvox, const double* map, const uint32_t* bin_mat,
                  int n_nodes, int n_bins, float* lut_rho, uint8_t* lut_mat, float* rho,
                  uint8_t* mat, uint32_t* rmax_bits, void* stream)
{
    hipLaunchKernelGGL(ct_lut_kernel, dim3(kCtLutSize / 256), dim3(256), 0, (hipStream_t)stream,
                       map, bin_mat, n_nodes, n_bins, lut_rho, lut_mat);
    if (status()) return -1;
    const size_t per = size_t(256) * kCtRun;
    const size_t blocks = std::min<size_t>((nvox + per - 1) / per, 16384);
    hipLaunchKernelGGL(ct_map_kernel, dim3(unsigned(blocks)), dim3(256), 0, (hipStream_t)stream,
                       hu, nvox, lut_rho, lut_mat, rho, mat, rmax_bits);
    return status();
}

}  // namespace omc
