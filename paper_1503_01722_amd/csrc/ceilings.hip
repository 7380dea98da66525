// ceilings.hip -- microbenchmarks of the MI355X ceilings the transport path is
// measured against: the plain-ALU lane-operation rate (non-packed FP32 FMA and
// 32-bit integer chains), an HBM stream, and device-scope FP64 atomic adds
// (the dose tally's one FP64 step, Sec. 2.2.2: an atomic dose counter) at
// random addresses over a footprint and on one contended address.
//
// Each entry point launches its kernel `reps` times on the null stream and
// returns the best launch time (HIP events) in *ms, with the work per launch
// in *work (lane operations, bytes or atomics). Built into its own library
// (libomc_ceilings.so): measurement, not part of the transport path.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

// Eight independent dependency chains per lane, each iteration one FMA per
// chain (8 lane-ops); the chains keep the VALU pipeline full without packed
// FP32 (disabled at compile time).
__global__ void __launch_bounds__(256) valu_fma_kernel(float* out, int iters, float a, float b)
{
    float x0 = threadIdx.x, x1 = x0 + 1, x2 = x0 + 2, x3 = x0 + 3;
    float x4 = x0 + 4, x5 = x0 + 5, x6 = x0 + 6, x7 = x0 + 7;
    for (int i = 0; i < iters; ++i) {
        x0 = __builtin_fmaf(x0, a, b);
        x1 = __builtin_fmaf(x1, a, b);
        x2 = __builtin_fmaf(x2, a, b);
        x3 = __builtin_fmaf(x3, a, b);
        x4 = __builtin_fmaf(x4, a, b);
        x5 = __builtin_fmaf(x5, a, b);
        x6 = __builtin_fmaf(x6, a, b);
        x7 = __builtin_fmaf(x7, a, b);
    }
    const float s = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
    if (s == 1234.5f) out[blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the chains live
}

// Full-rate 32-bit integer work: an add and a rotate-free shift-xor per
// chain and iteration (two lane-ops), eight chains.
__global__ void __launch_bounds__(256) valu_int_kernel(uint32_t* out, int iters, uint32_t a,
                                                       uint32_t b)
{
    uint32_t x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = threadIdx.x + 977u * k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = (x[k] + a) ^ b;
        a += 1u;
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s ^= x[k];
    if (s == 0x12345678u) out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Copy n 16-byte elements: n * 32 bytes of HBM traffic.
__global__ void __launch_bounds__(256) stream_copy_kernel(const float4* __restrict__ src,
                                                          float4* __restrict__ dst, size_t n)
{
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// FP64 atomic adds (no return: global_atomic_add_f64) at addresses drawn
// uniformly over `footprint` doubles; per_thread adds per work-item.
__global__ void __launch_bounds__(256) atomic_random_kernel(double* grid, uint32_t footprint,
                                                            int per_thread, uint32_t seed)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t h = mix32(t ^ seed);
    for (int i = 0; i < per_thread; ++i) {
        h = mix32(h + 0x9E3779B9u);
        unsafeAtomicAdd(&grid[h % footprint], 1.0);
    }
}

// Every add of a work-group's waves to one of `hot` addresses (hot = 1: a
// single contended voxel).
__global__ void __launch_bounds__(256) atomic_hot_kernel(double* grid, uint32_t hot,
                                                         int per_thread)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = 0; i < per_thread; ++i) unsafeAtomicAdd(&grid[(t + i) % hot], 1.0);
}

template <typename F>
int time_best(int reps, double* ms, F&& launch)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -3;
    double best = 1e30;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(a, nullptr);
        launch();
        (void)hipEventRecord(b, nullptr);
        if (hipEventSynchronize(b) != hipSuccess) {
            best = -1;
            break;
        }
        float t = 0;
        (void)hipEventElapsedTime(&t, a, b);
        if (t < best) best = t;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (best < 0 || hipGetLastError() != hipSuccess) return -3;
    *ms = best;
    return 0;
}

int cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return n;
}

}  // namespace

extern "C" {

// kind 0: FP32 FMA chains (1 lane-op per FMA); 1: integer add + xor chains
// (2 lane-ops per chain and iteration). blocks_per_cu work-groups of 256.
int omc_ceil_valu(int kind, int blocks_per_cu, int iters, int reps, double* ms, double* work)
{
    const int n_cu = cus();
    if (n_cu <= 0 || blocks_per_cu < 1 || blocks_per_cu > 64 || iters < 1 || reps < 1 || !ms ||
        !work)
        return -1;
    const int grid = n_cu * blocks_per_cu;
    void* out = nullptr;
    if (hipMalloc(&out, size_t(grid) * 256 * 4) != hipSuccess) return -2;
    int rc;
    if (kind == 0) {
        rc = time_best(reps, ms, [&] {
            hipLaunchKernelGGL(valu_fma_kernel, dim3(grid), dim3(256), 0, nullptr,
                               static_cast<float*>(out), iters, 0.999f, 0.001f);
        });
        *work = double(grid) * 256.0 * iters * 8.0;
    } else {
        rc = time_best(reps, ms, [&] {
            hipLaunchKernelGGL(valu_int_kernel, dim3(grid), dim3(256), 0, nullptr,
                               static_cast<uint32_t*>(out), iters, 0x9E3779B1u, 0x7F4A7C15u);
        });
        *work = double(grid) * 256.0 * iters * 8.0 * 2.0;
    }
    (void)hipFree(out);
    return rc;
}

// Copy of `bytes` (rounded down to 16) between two device buffers; work =
// bytes read + bytes written.
int omc_ceil_stream(size_t bytes, int reps, double* ms, double* work)
{
    const int n_cu = cus();
    const size_t n = bytes / 16;
    if (n_cu <= 0 || n == 0 || reps < 1 || !ms || !work) return -1;
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, n * 16) != hipSuccess) return -2;
    if (hipMalloc(&b, n * 16) != hipSuccess) {
        (void)hipFree(a);
        return -2;
    }
    (void)hipMemset(a, 0, n * 16);
    const int rc = time_best(reps, ms, [&] {
        hipLaunchKernelGGL(stream_copy_kernel, dim3(n_cu * 8), dim3(256), 0, nullptr,
                           static_cast<const float4*>(a), static_cast<float4*>(b), n);
    });
    *work = 2.0 * double(n) * 16.0;
    (void)hipFree(a);
    (void)hipFree(b);
    return rc;
}

// FP64 atomic adds: mode 0 at uniform random addresses over `footprint`
// doubles, mode 1 onto `footprint` hot addresses (1 = one contended voxel).
// threads work-items (multiple of 256) with per_thread adds each.
int omc_ceil_atomic(int mode, uint32_t footprint, uint32_t threads, int per_thread, int reps,
                    double* ms, double* work)
{
    if (footprint == 0 || threads == 0 || threads % 256 || per_thread < 1 || reps < 1 || !ms ||
        !work || (mode != 0 && mode != 1))
        return -1;
    double* g = nullptr;
    if (hipMalloc(&g, size_t(footprint) * sizeof(double)) != hipSuccess) return -2;
    (void)hipMemset(g, 0, size_t(footprint) * sizeof(double));
    int rc;
    if (mode == 0)
        rc = time_best(reps, ms, [&] {
            hipLaunchKernelGGL(atomic_random_kernel, dim3(threads / 256), dim3(256), 0, nullptr, g,
                               footprint, per_thread, 12345u);
        });
    else
        rc = time_best(reps, ms, [&] {
            hipLaunchKernelGGL(atomic_hot_kernel, dim3(threads / 256), dim3(256), 0, nullptr, g,
                               footprint, per_thread);
        });
    *work = double(threads) * per_thread;
    (void)hipFree(g);
    return rc;
}

}  // extern "C"
