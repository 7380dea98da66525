// kernels_f32.hip -- production transport in FP32 (FP64 tally), plus the
// precision-independent helper kernels: batch fold, queue control, zero fill,
// statistics reduce, batched-beamlet compaction and the Philox debug kernel.
#include "kernels_impl.hpp"

namespace omc {

template struct Launch<float>;

// dose_v = sum_b E_vb / (rho_v V N); dose2_v = sum_b (E_vb / (rho_v V N_b))^2,
// batches in order (Sec. 3.1 reports sigma_D per voxel; batch method); E_vb is
// the sum, in order, of the batch's private copies.
struct BatchSizes {
    double nb[64];
};

__global__ void __launch_bounds__(256)
fold_kernel(const double* __restrict__ grid, const float* __restrict__ rho, size_t nvox, int B,
            int K, BatchSizes nbs, double V, double N, double* __restrict__ dose,
            double* __restrict__ dose2)
{
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nvox; v += stride) {
        const double mV = double(rho[v]) * V;
        double d = 0.0, d2 = 0.0;
        for (int b = 0; b < B; ++b) {
            if (!(nbs.nb[b] > 0.0)) continue;
            const double* g = grid + size_t(b) * size_t(K) * nvox + v;
            double e = g[0];
            for (int k = 1; k < K; ++k) e += g[size_t(k) * nvox];
            d += e / (mV * N);
            const double db = e / (mV * nbs.nb[b]);
            d2 += db * db;
        }
        dose[v] = d;
        dose2[v] = d2;
    }
}

int launch_fold(const double* grid, const float* rho, size_t nvox, int B, int copies,
                const double* nb, double V, double n_total, double* dose, double* dose2,
                void* stream)
{
    if (B < 1 || B > 64 || copies < 1) return -1;
    BatchSizes nbs{};
    for (int b = 0; b < B; ++b) nbs.nb[b] = nb[b];
    const int block = 256;
    size_t blocks = (nvox + block - 1) / block;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fold_kernel, dim3(unsigned(blocks)), dim3(block), 0, (hipStream_t)stream,
                       grid, rho, nvox, B, copies, nbs, V, n_total, dose, dose2);
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

// Ordered source: each energy group's first slot after the groups above it
// (group 0 the highest energies), and the counts cleared for the next chunk.
__global__ void source_scan_kernel(uint32_t* order)
{
    if (threadIdx.x == 0) {
        uint32_t acc = 0u;
        for (int g = 0; g < kSrcGroups; ++g) {
            order[kSrcGroups + g] = acc;
            acc += order[g];
            order[g] = 0u;
        }
    }
}

int launch_source_scan(uint32_t* order, void* stream)
{
    hipLaunchKernelGGL(source_scan_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, order);
    return detail::launch_status();
}

// ctrl layout: [2q] count and [2q+1] head of queue q (0, 1 photons; 2, 3
// electrons), [8] overflow flag, [9] longest particle, [10] electron and [11]
// photon queue high-water marks.
__global__ void queue_commit_kernel(uint32_t* ctrl, int q, uint32_t add)
{
    if (threadIdx.x == 0) {
        const uint32_t n = ctrl[2 * q] + add;
        ctrl[2 * q] = n;
        uint32_t& hwm = ctrl[q < 2 ? 11 : 10];
        if (n > hwm) hwm = n;
    }
}

int launch_queue_commit(uint32_t* ctrl, int which, uint32_t add, void* stream)
{
    if (which < 0 || which > 3) return -1;
    hipLaunchKernelGGL(queue_commit_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, ctrl,
                       which, add);
    return detail::launch_status();
}

__global__ void __launch_bounds__(256) zero_kernel(unsigned long long* p, size_t n)
{
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

int launch_zero(void* p, size_t n_words, void* stream)
{
    if (n_words == 0) return 0;
    size_t blocks = (n_words + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(zero_kernel, dim3(unsigned(blocks)), dim3(256), 0, (hipStream_t)stream,
                       static_cast<unsigned long long*>(p), n_words);
    return detail::launch_status();
}

// ------------------------------------------------------- beamlet compaction
// Dose of one cell of beam b: E * scale_b / rho_v (MeV/g per history).
__device__ __forceinline__ float cell_dose(double e, double scale, float rho)
{
    return float(e * scale / double(rho));
}

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t x, uint32_t* s_w)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += uint32_t(__shfl_xor(int(x), off));
    __syncthreads();
    if (__lane_id() == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) t += s_w[w];
    return t;
}

// per-beam maximum dose (non-negative float bits order as integers)
__global__ void __launch_bounds__(256)
beam_max_kernel(const double* __restrict__ grid, const float* __restrict__ rho, size_t nvox,
                const double* __restrict__ scale, float* __restrict__ dmax)
{
    const int b = blockIdx.y;
    const double* g = grid + size_t(b) * nvox;
    const double sc = scale[b];
    float m = 0.0f;
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nvox; v += stride) {
        const double e = g[v];
        if (e != 0.0) m = fmaxf(m, cell_dose(e, sc, rho[v]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (__lane_id() == 0 && m > 0.0f)
        atomicMax(reinterpret_cast<unsigned int*>(dmax + b), __float_as_uint(m));
}

int launch_beam_max(const double* grid, const float* rho, size_t nvox, int n_beams,
                    const double* scale, float* dmax, void* stream)
{
    size_t bx = (nvox + 255) / 256;
    if (bx > 512) bx = 512;
    hipLaunchKernelGGL(beam_max_kernel, dim3(unsigned(bx), unsigned(n_beams)), dim3(256), 0,
                       (hipStream_t)stream, grid, rho, nvox, scale, dmax);
    return detail::launch_status();
}

// A work-group of 256 owns one tile of kCompactTile voxels of one beam; its
// thread t looks at voxels tile_start + k * 256 + t, k = 0..7.
constexpr int kPerThread = kCompactTile / 256;

__global__ void __launch_bounds__(256)
compact_count_kernel(const double* __restrict__ grid, const float* __restrict__ rho, size_t nvox,
                     const double* __restrict__ scale, const float* __restrict__ thr,
                     uint32_t* __restrict__ tile_cnt)
{
    __shared__ uint32_t s_w[4];
    const int b = blockIdx.y;
    const size_t v0 = size_t(blockIdx.x) * kCompactTile;
    const double* g = grid + size_t(b) * nvox;
    const double sc = scale[b];
    const float th = thr[b];
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const size_t v = v0 + size_t(k) * 256 + threadIdx.x;
        if (v < nvox) {
            const double e = g[v];
            if (e != 0.0 && cell_dose(e, sc, rho[v]) > th) ++n;
        }
    }
    n = block_sum_u32(n, s_w);
    if (threadIdx.x == 0) tile_cnt[size_t(b) * gridDim.x + blockIdx.x] = n;
}

int launch_compact_count(const double* grid, const float* rho, size_t nvox, int n_beams,
                         const double* scale, const float* thr, uint32_t* tile_cnt, void* stream)
{
    const size_t tiles = (nvox + kCompactTile - 1) / kCompactTile;
    if (tiles > 0x7fffffff || n_beams > 65535) return -1;
    hipLaunchKernelGGL(compact_count_kernel, dim3(unsigned(tiles), unsigned(n_beams)), dim3(256),
                       0, (hipStream_t)stream, grid, rho, nvox, scale, thr, tile_cnt);
    return detail::launch_status();
}

__global__ void __launch_bounds__(256)
compact_write_kernel(const double* __restrict__ grid, const float* __restrict__ rho, size_t nvox,
                     const double* __restrict__ scale, const float* __restrict__ thr,
                     const uint64_t* __restrict__ tile_off, uint64_t nnz,
                     uint32_t* __restrict__ voxel, float* __restrict__ dose)
{
    __shared__ uint32_t s_w[4];
    const int b = blockIdx.y;
    const size_t v0 = size_t(blockIdx.x) * kCompactTile;
    const double* g = grid + size_t(b) * nvox;
    const double sc = scale[b];
    const float th = thr[b];
    uint64_t out = tile_off[size_t(b) * gridDim.x + blockIdx.x];
    const int wave = threadIdx.x >> 6;
    for (int k = 0; k < kPerThread; ++k) {
        const size_t v = v0 + size_t(k) * 256 + threadIdx.x;
        float d = 0.0f;
        bool keep = false;
        if (v < nvox) {
            const double e = g[v];
            if (e != 0.0) {
                d = cell_dose(e, sc, rho[v]);
                keep = d > th;
            }
        }
        const uint64_t m = __ballot(keep);
        __syncthreads();
        if (__lane_id() == 0) s_w[wave] = uint32_t(__popcll(m));
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wave) before += s_w[w];
            total += s_w[w];
        }
        if (keep) {
            const uint64_t pos =
                out + before + uint32_t(__popcll(m & ((uint64_t(1) << __lane_id()) - 1)));
            if (pos < nnz) {  // the count pass decided the same way; never past the rows
                voxel[pos] = uint32_t(v);
                dose[pos] = d;
            }
        }
        out += total;
    }
}

int launch_compact_write(const double* grid, const float* rho, size_t nvox, int n_beams,
                         const double* scale, const float* thr, const uint64_t* tile_off,
                         uint64_t nnz, uint32_t* voxel, float* dose, void* stream)
{
    const size_t tiles = (nvox + kCompactTile - 1) / kCompactTile;
    if (tiles > 0x7fffffff || n_beams > 65535) return -1;
    hipLaunchKernelGGL(compact_write_kernel, dim3(unsigned(tiles), unsigned(n_beams)), dim3(256),
                       0, (hipStream_t)stream, grid, rho, nvox, scale, thr, tile_off, nnz, voxel,
                       dose);
    return detail::launch_status();
}

// Exclusive scan in three launches: 1024-count segments scanned by one
// work-group each (segment totals to tmp), one work-group scanning the segment
// totals, then the segment offsets added.
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(x, off);
        if (int(__lane_id()) >= off) x += y;
    }
    return x;
}

// block-wide exclusive scan of one value per thread (256 threads); *total gets the sum
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t x, uint64_t* s_w, uint64_t* total)
{
    const uint64_t inc = wave_incl_scan(x);
    __syncthreads();
    if (__lane_id() == 63) s_w[threadIdx.x >> 6] = inc;
    __syncthreads();
    uint64_t before = 0, t = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < int(threadIdx.x >> 6)) before += s_w[w];
        t += s_w[w];
    }
    *total = t;
    return before + inc - x;
}

__global__ void __launch_bounds__(256)
scan_segments_kernel(const uint32_t* __restrict__ in, uint64_t* __restrict__ out, size_t n,
                     uint64_t* __restrict__ seg)
{
    __shared__ uint64_t s_w[4];
    const size_t i0 = size_t(blockIdx.x) * 1024 + size_t(threadIdx.x) * 4;
    uint64_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = i0 + k < n ? in[i0 + k] : 0u;
        sum += v[k];
    }
    uint64_t total;
    uint64_t pre = block_excl_scan(sum, s_w, &total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (i0 + k < n) out[i0 + k] = pre;
        pre += v[k];
    }
    if (threadIdx.x == 0) seg[blockIdx.x] = total;
}

__global__ void __launch_bounds__(256) scan_top_kernel(uint64_t* seg, size_t n_seg)
{
    __shared__ uint64_t s_w[4];
    uint64_t carry = 0;
    for (size_t base = 0; base < n_seg; base += 256) {
        const size_t i = base + threadIdx.x;
        const uint64_t x = i < n_seg ? seg[i] : 0u;
        uint64_t total;
        const uint64_t pre = block_excl_scan(x, s_w, &total);
        if (i < n_seg) seg[i] = carry + pre;
        carry += total;
    }
    if (threadIdx.x == 0) seg[n_seg] = carry;
}

__global__ void __launch_bounds__(256)
scan_add_kernel(uint64_t* __restrict__ out, size_t n, const uint64_t* __restrict__ seg,
                size_t n_seg)
{
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] += seg[i / 1024];
    if (i == 0) out[n] = seg[n_seg];
}

int launch_scan(const uint32_t* in, uint64_t* out, size_t n, uint64_t* tmp, void* stream)
{
    if (n == 0) return -1;
    const size_t n_seg = (n + 1023) / 1024;
    if (n_seg > 0x7fffffff) return -1;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(scan_segments_kernel, dim3(unsigned(n_seg)), dim3(256), 0, s, in, out, n,
                       tmp);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(256), 0, s, tmp, n_seg);
    hipLaunchKernelGGL(scan_add_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, out, n,
                       tmp, n_seg);
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

__global__ void __launch_bounds__(256)
check_records_kernel(const float* rec, uint32_t n, double ehi, uint32_t* out)
{
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= n) return;
    const float* q = rec + 8 * size_t(k);
    bool ok = q[0] > 0.0f && double(q[0]) < ehi;
    for (int j = 1; j < 7; ++j) ok = ok && __builtin_isfinite(q[j]);
    // float squares are exact in double, so the sum matches the host's
    const double n2 = double(q[4]) * q[4] + double(q[5]) * q[5] + double(q[6]) * q[6];
    if (!ok || !(n2 > 1e-12)) {
        atomicAdd(out, 1u);
        atomicMin(out + 1, k);
    }
}

int launch_check_records(const float* rec, uint32_t n, double ehi, uint32_t* out, void* stream)
{
    const unsigned grid = (n + 255) / 256;
    hipLaunchKernelGGL(check_records_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, rec,
                       n, ehi, out);
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
