// kernels_f32.hip -- production transport in FP32 (FP64 tally), plus the
// precision-independent helper kernels: batch fold, queue reset and the Philox
// debug kernel.
#include "kernels_impl.hpp"

namespace omc {

template struct Launch<float>;

// dose_v = sum_b E_vb / (rho_v V N); dose2_v = sum_b (E_vb / (rho_v V N_b))^2,
// batches in order (Sec. 3.1 reports sigma_D per voxel; batch method).
struct BatchSizes {
    double nb[64];
};

__global__ void __launch_bounds__(256)
fold_kernel(const double* __restrict__ grid, const float* __restrict__ rho, size_t nvox, int B,
            BatchSizes nbs, double V, double N, double* __restrict__ dose,
            double* __restrict__ dose2)
{
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nvox; v += stride) {
        const double mV = double(rho[v]) * V;
        double d = 0.0, d2 = 0.0;
        for (int b = 0; b < B; ++b) {
            if (!(nbs.nb[b] > 0.0)) continue;
            const double e = grid[size_t(b) * nvox + v];
            d += e / (mV * N);
            const double db = e / (mV * nbs.nb[b]);
            d2 += db * db;
        }
        dose[v] = d;
        dose2[v] = d2;
    }
}

int launch_fold(const double* grid, const float* rho, size_t nvox, int B, const double* nb,
                double V, double n_total, double* dose, double* dose2, void* stream)
{
    if (B < 1 || B > 64) return -1;
    BatchSizes nbs{};
    for (int b = 0; b < B; ++b) nbs.nb[b] = nb[b];
    const int block = 256;
    size_t blocks = (nvox + block - 1) / block;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fold_kernel, dim3(unsigned(blocks)), dim3(block), 0, (hipStream_t)stream,
                       grid, rho, nvox, B, nbs, V, n_total, dose, dose2);
    return detail::launch_status();
}

// Clear {count, head} of the queues selected by mask (bit q -> queue q).
__global__ void queue_reset_kernel(uint32_t* ctrl, int mask)
{
    const int q = threadIdx.x;
    if (q < 4 && (mask >> q) & 1) {
        ctrl[2 * q] = 0u;
        ctrl[2 * q + 1] = 0u;
    }
}

int launch_queue_reset(uint32_t* ctrl, int mask, void* stream)
{
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, ctrl, mask);
    return detail::launch_status();
}

// Column sums of the statistics buffer into row 0: one work-group per column,
// 256 threads striding over the rows, then a tree in LDS.
__global__ void __launch_bounds__(256) stats_reduce_kernel(unsigned long long* counters,
                                                          double* energies, uint32_t n_rows)
{
    __shared__ unsigned long long su[256];
    __shared__ double sd[256];
    const int col = blockIdx.x;
    const bool is_count = col < kNumCounters;
    const int j = is_count ? col : col - kNumCounters;
    unsigned long long u = 0;
    double v = 0.0;
    for (uint32_t r = threadIdx.x; r < n_rows; r += blockDim.x) {
        if (is_count) u += counters[size_t(r) * kNumCounters + j];
        else v += energies[size_t(r) * kNumEnergies + j];
    }
    su[threadIdx.x] = u;
    sd[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) {
            su[threadIdx.x] += su[threadIdx.x + s];
            sd[threadIdx.x] += sd[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (is_count) counters[j] = su[0];
        else energies[j] = sd[0];
    }
}

int launch_stats_reduce(unsigned long long* counters, double* energies, uint32_t n_rows,
                        void* stream)
{
    hipLaunchKernelGGL(stats_reduce_kernel, dim3(kNumCounters + kNumEnergies), dim3(256), 0,
                       (hipStream_t)stream, counters, energies, n_rows);
    return detail::launch_status();
}

__global__ void philox_debug_kernel(uint32_t seed, uint32_t h, uint32_t qlo, uint32_t qhi,
                                    uint32_t n0, uint32_t nblocks, uint32_t* out)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    uint32_t o0, o1, o2, o3;
    Stream::block(n0 + b, qlo, qhi, 0u, seed, h, o0, o1, o2, o3);
    out[4 * size_t(b) + 0] = o0;
    out[4 * size_t(b) + 1] = o1;
    out[4 * size_t(b) + 2] = o2;
    out[4 * size_t(b) + 3] = o3;
}

int launch_philox_debug(uint32_t seed, uint32_t h, uint64_t q, uint32_t n0, uint32_t nblocks,
                        uint32_t* out, void* stream)
{
    const unsigned grid = (nblocks + 255) / 256;
    hipLaunchKernelGGL(philox_debug_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, seed,
                       h, uint32_t(q), uint32_t(q >> 32), n0, nblocks, out);
    return detail::launch_status();
}

}  // namespace omc
