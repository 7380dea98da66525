// dn_kernels.hip -- gfx950 kernels of the learned dose denoiser: implicit-GEMM
// convolutions on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulate) for the forward pass, the input gradient and the weight
// gradient, plus the elementwise, loss and optimiser kernels.
//
// Lane layout of v_mfma_f32_16x16x32_bf16 (64 lanes, r = lane % 16, g = lane /
// 16): the A operand of lane (r, g) is A[r][8g .. 8g+7], the B operand is
// B[8g .. 8g+7][r], and the four FP32 results are D[4g + i][r], i = 0..3.
#include <hip/hip_runtime.h>

#include "dn.hpp"

namespace dn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

int status() { return hipGetLastError() == hipSuccess ? 0 : -1; }

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// round to nearest, ties to even (finite values)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// Input voxel read by output voxel (z, y, x) at tap t, or -1 outside the volume.
template <int GEOM>
__device__ __forceinline__ long long window_voxel(const Dims& in, int z, int y, int x, int t)
{
    int iz, iy, ix;
    if (GEOM == G_CONV3) {
        iz = z + t / 9 - 1;
        iy = y + (t / 3) % 3 - 1;
        ix = x + t % 3 - 1;
    } else {  // G_DOWN
        iz = 2 * z + (t >> 2);
        iy = 2 * y + ((t >> 1) & 1);
        ix = 2 * x + (t & 1);
    }
    if (iz < 0 || iy < 0 || ix < 0 || iz >= in.nz || iy >= in.ny || ix >= in.nx) return -1;
    return ((long long)iz * in.ny + iy) * in.nx + ix;
}

// Output voxel 2 v + t of input voxel (z, y, x) in a volume of dims `out`.
__device__ __forceinline__ size_t up_voxel(const Dims& out, int z, int y, int x, int t)
{
    return (size_t(2 * z + (t >> 2)) * out.ny + size_t(2 * y + ((t >> 1) & 1))) * out.nx +
           size_t(2 * x + (t & 1));
}

__device__ __forceinline__ void decompose(size_t m, const Dims& d, int& z, int& y, int& x)
{
    x = int(m % size_t(d.nx));
    const size_t q = m / size_t(d.nx);
    y = int(q % size_t(d.ny));
    z = int(q / size_t(d.ny));
}

struct ConvParams {
    const uint16_t* x0;
    const uint16_t* x1;
    int c0, c1;
    Dims in, out;
    const uint16_t* packed;
    int K, N, kblocks;
    size_t M;  // GEMM rows
    ConvOut o;
};

// One work-group: 4 waves x 64 rows (4 row tiles of 16 per wave) and NT
// column tiles of 16. The A operand is gathered straight from the
// channels-last input (16 bytes per lane per row tile and reduction block;
// neighbouring taps hit the same cache lines), B from the packed weights.
template <int GEOM, int NT>
__global__ void __launch_bounds__(256) conv_kernel(ConvParams p)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const size_t row0 = size_t(blockIdx.x) * 256 + size_t(wave) * 64;
    const int nt0 = blockIdx.y * NT;
    const int cin = p.c0 + p.c1;
    const Dims rows = GEOM == G_UP ? p.in : p.out;

    int rz[4], ry[4], rx[4];
    bool rv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const size_t m = row0 + size_t(16 * s + r);
        rv[s] = m < p.M;
        decompose(rv[s] ? m : 0, rows, rz[s], ry[s], rx[s]);
    }
    f32x4 acc[4][NT];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[s][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    const uint4* bsrc = reinterpret_cast<const uint4*>(p.packed);
    for (int kb = 0; kb < p.kblocks; ++kb) {
        const int k0 = kb * 32 + g * 8;
        const bool kv = k0 < p.K;
        int t = 0, ci = k0;
        if (GEOM != G_UP) {
            t = k0 / cin;
            ci = k0 - t * cin;
        }
        bf16x8 a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            uint4 raw = {0u, 0u, 0u, 0u};
            if (kv && rv[s]) {
                long long v;
                if (GEOM == G_UP) v = ((long long)rz[s] * rows.ny + ry[s]) * rows.nx + rx[s];
                else v = window_voxel<GEOM>(p.in, rz[s], ry[s], rx[s], t);
                if (v >= 0) {
                    const uint16_t* src = ci < p.c0 ? p.x0 + size_t(v) * p.c0 + ci
                                                    : p.x1 + size_t(v) * p.c1 + (ci - p.c0);
                    raw = *reinterpret_cast<const uint4*>(src);
                }
            }
            a[s] = as_bf16x8(raw);
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const bf16x8 b = as_bf16x8(bsrc[(size_t(nt0 + n) * p.kblocks + kb) * 64 + lane]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[s][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], b, acc[s][n], 0, 0, 0);
        }
    }

    // epilogue: lane (r, g) holds rows 4g + i, column r of every tile
    const int n_up = GEOM == G_UP ? p.N / 8 : p.N;  // channels of the output volume
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const size_t m = row0 + size_t(16 * s + 4 * g + i);
            if (m >= p.M) continue;
            int z = 0, y = 0, x = 0;
            if (GEOM == G_UP) decompose(m, rows, z, y, x);
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int col = (nt0 + n) * 16 + r;
                float v = acc[s][n][i];
                size_t ov = m;
                int ch = col;
                if (GEOM == G_UP) {
                    const int t = col / n_up;
                    ch = col - t * n_up;
                    ov = up_voxel(p.out, z, y, x, t);
                }
                if (p.o.y) {
                    if (p.o.bias) v += p.o.bias[ch];
                    if (p.o.relu) v = fmaxf(v, 0.f);
                    p.o.y[ov * size_t(n_up) + ch] = f2bf(v);
                } else if (ch < p.o.split) {
                    float* d = p.o.g0 + ov * size_t(p.o.split) + ch;
                    *d = p.o.acc0 ? *d + v : v;
                } else {
                    const int w1 = n_up - p.o.split;
                    float* d = p.o.g1 + ov * size_t(w1) + (ch - p.o.split);
                    *d = p.o.acc1 ? *d + v : v;
                }
            }
        }
    }
}

// ------------------------------------------------ 3x3x3 convolution, LDS tile
// The same GEMM as conv_kernel<G_CONV3, NT> for inputs of 8 to 96 channels,
// with the input staged once per work-group instead of gathered per tap. A
// work-group owns an output block of BZ x 4 x 16 voxels (x fastest): it
// copies the block's input with its one-voxel halo, (BZ+2) x 6 x 18 voxels,
// into LDS (channels-last, voxel pitch an odd number of 16-byte chunks so
// that 16 consecutive voxels fall in distinct bank groups; zeros outside the
// volume), then each of its four waves computes RS = BZ row tiles (a row
// tile is 16 voxels along x at one (z, y); a wave's tiles are consecutive in
// y). With the channel count a compile-time constant, the LDS offset of every
// (reduction block, lane group) is a constant and the row tile's an
// immediate. The reduction order over (tap, channel) blocks of 32 is that of
// conv_kernel, so both give the same sums.
constexpr int kTileX = 16;

template <int CIN>
struct TileShape {
    // 16 row tiles of 4 per wave up to 48 channels, 8 of 2 per wave above
    static constexpr int BZ = CIN <= 48 ? 4 : 2;
    static constexpr int BY = 4;
    static constexpr int RS = BZ * BY / 4;  // row tiles per wave
    static constexpr int SY = BY + 2, SX = kTileX + 2;
    static constexpr int PC = (CIN / 8) | 1;  // 16-byte chunks per staged voxel
    static constexpr int K = 27 * CIN;
    static constexpr int KB = (K + 31) / 32;
    static constexpr size_t lds = size_t(BZ + 2) * SY * SX * PC * 16;
    // LDS chunk offset of reduction index k0 (a multiple of 8) from the
    // haloed block's origin: tap (dz, dy, dx) reads voxel (z+dz, y+dy, x+dx)
    static constexpr int chunk(int k0)
    {
        if (k0 >= K) return 0;
        const int t = k0 / CIN, ci = k0 % CIN;
        return (((t / 9) * SY + (t / 3) % 3) * SX + t % 3) * PC + ci / 8;
    }
};

template <int NT, int CIN>
__global__ void __launch_bounds__(256) conv3_tile_kernel(ConvParams p)
{
    using S = TileShape<CIN>;
    constexpr int BZ = S::BZ, BY = S::BY, RS = S::RS, SY = S::SY, SX = S::SX, PC = S::PC;
    constexpr int KB = S::KB;
    static_assert(BY % RS == 0, "a wave's row tiles share z");
    extern __shared__ __align__(16) uint4 tile[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int nxt = (p.out.nx + kTileX - 1) / kTileX;
    const int x0 = (int(blockIdx.x) % nxt) * kTileX;
    const int y0 = (int(blockIdx.x) / nxt) * BY;
    const int z0 = int(blockIdx.y) * BZ;
    const int nt0 = int(blockIdx.z) * NT;

    // stage: piece q = (voxel of the haloed block, chunk of 8 channels); each
    // thread issues kSB loads before it writes any, so they are in flight together
    constexpr int CG = CIN / 8;
    constexpr int PIECES = (BZ + 2) * SY * SX * CG;
    constexpr int kSB = 8;
    for (int q0 = threadIdx.x; q0 < PIECES; q0 += 256 * kSB) {
        uint4 raw[kSB];
#pragma unroll
        for (int u = 0; u < kSB; ++u) {
            const int q = q0 + 256 * u;
            raw[u] = uint4{0u, 0u, 0u, 0u};
            if (q < PIECES) {
                const int c = q % CG;
                const int v = q / CG;
                const int lx = v % SX, ly = (v / SX) % SY, lz = v / (SX * SY);
                const int ix = x0 + lx - 1, iy = y0 + ly - 1, iz = z0 + lz - 1;
                if (ix >= 0 && iy >= 0 && iz >= 0 && ix < p.in.nx && iy < p.in.ny &&
                    iz < p.in.nz) {
                    const size_t gv = (size_t(iz) * p.in.ny + iy) * p.in.nx + ix;
                    const int ci = c * 8;
                    const uint16_t* src =
                        ci < p.c0 ? p.x0 + gv * p.c0 + ci : p.x1 + gv * p.c1 + (ci - p.c0);
                    raw[u] = *reinterpret_cast<const uint4*>(src);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kSB; ++u) {
            const int q = q0 + 256 * u;
            if (q < PIECES) tile[(q / CG) * PC + q % CG] = raw[u];
        }
    }
    __syncthreads();

    const uint4* bsrc = reinterpret_cast<const uint4*>(p.packed);
    // weight fragments in groups of KU reduction blocks: the next group is
    // loaded while the current group's products run
    constexpr int KU = NT <= 2 ? 4 : 2;
    auto load_b = [&](bf16x8 (&dst)[KU][NT], int kb0) {
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int kb = kb0 + u;
                const uint4 raw = kb < KB ? bsrc[(size_t(nt0 + n) * KB + kb) * 64 + lane]
                                          : uint4{0u, 0u, 0u, 0u};
                dst[u][n] = as_bf16x8(raw);
            }
    };
    {
        const int rt0 = wave * RS;
        const int lb = (((rt0 / BY) * SY + rt0 % BY) * SX + r) * PC;  // row tile s: + s*SX*PC
        f32x4 acc[RS][NT];
#pragma unroll
        for (int s = 0; s < RS; ++s)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[s][n] = f32x4{0.f, 0.f, 0.f, 0.f};
        bf16x8 b[KU][NT], bn[KU][NT];
        load_b(b, 0);
#pragma unroll
        for (int kb0 = 0; kb0 < KB; kb0 += KU) {
            if (kb0 + KU < KB) load_b(bn, kb0 + KU);
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int kb = kb0 + u;
                if (kb >= KB) break;
                const int o0 = S::chunk(kb * 32), o1 = S::chunk(kb * 32 + 8);
                const int o2 = S::chunk(kb * 32 + 16), o3 = S::chunk(kb * 32 + 24);
                const int off = lb + (g == 0 ? o0 : g == 1 ? o1 : g == 2 ? o2 : o3);
                const bool kv = kb * 32 + g * 8 < S::K;  // false only in the last block
                bf16x8 a[RS];
#pragma unroll
                for (int s = 0; s < RS; ++s) {
                    uint4 raw = tile[off + s * SX * PC];
                    if (!kv) raw = uint4{0u, 0u, 0u, 0u};
                    a[s] = as_bf16x8(raw);
                }
#pragma unroll
                for (int n = 0; n < NT; ++n)
#pragma unroll
                    for (int s = 0; s < RS; ++s)
                        acc[s][n] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], b[u][n], acc[s][n], 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < KU; ++u)
#pragma unroll
                for (int n = 0; n < NT; ++n) b[u][n] = bn[u][n];
        }
        // epilogue: lane (r, g) holds voxels x0 + 4g + i of each row tile, column r
#pragma unroll
        for (int s = 0; s < RS; ++s) {
            const int rt = rt0 + s;
            const int z = z0 + rt / BY, y = y0 + rt % BY;
            if (z >= p.out.nz || y >= p.out.ny) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = x0 + 4 * g + i;
                if (x >= p.out.nx) continue;
                const size_t ov = (size_t(z) * p.out.ny + y) * p.out.nx + x;
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const int ch = (nt0 + n) * 16 + r;
                    float v = acc[s][n][i];
                    if (p.o.y) {
                        if (p.o.bias) v += p.o.bias[ch];
                        if (p.o.relu) v = fmaxf(v, 0.f);
                        p.o.y[ov * size_t(p.N) + ch] = f2bf(v);
                    } else if (ch < p.o.split) {
                        float* d = p.o.g0 + ov * size_t(p.o.split) + ch;
                        *d = p.o.acc0 ? *d + v : v;
                    } else {
                        const int w1 = p.N - p.o.split;
                        float* d = p.o.g1 + ov * size_t(w1) + (ch - p.o.split);
                        *d = p.o.acc1 ? *d + v : v;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------ weight gradient
constexpr int kWRows = 128;    // rows staged per step
constexpr int kWPitch = 136;   // LDS row pitch in BF16 (272 bytes: 16-byte aligned rows)

struct WgradParams {
    const uint16_t* x0;
    const uint16_t* x1;
    int c0, c1;
    Dims in, out;
    const uint16_t* g;
    int cout, cin_log;
    float* gw;
    float* gb;
    size_t M;            // rows (output voxels; input voxels for G_UP)
    size_t rows_per_block;
};

// One work-group: one tap (blockIdx.y) and a range of rows. Each step stages
// 128 rows of the gathered input and of the output gradient transposed into
// LDS ([channel][row]); wave w then multiplies rows 32w .. 32w+31 for every
// (input-channel tile, output-channel tile): D[ci][co] += A^T[ci][rows]
// G[rows][co]. The four waves' partial tiles are added to gw with FP32
// atomics at the end.
template <int GEOM, int TI, int TJ>
__global__ void __launch_bounds__(256) wgrad_kernel(WgradParams p)
{
    extern __shared__ __align__(16) uint16_t lds[];
    uint16_t* la = lds;                          // [TI*16][kWPitch]
    uint16_t* lg = lds + TI * 16 * kWPitch;      // [TJ*16][kWPitch]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int t = blockIdx.y;
    const int cin = p.c0 + p.c1;
    const Dims rows = GEOM == G_UP ? p.in : p.out;
    const size_t m_begin = size_t(blockIdx.x) * p.rows_per_block;
    size_t m_end = m_begin + p.rows_per_block;
    if (m_end > p.M) m_end = p.M;

    // channel rows beyond cin stay zero
    for (int i = threadIdx.x; i < (TI * 16 - cin) * kWPitch; i += 256)
        la[cin * kWPitch + i] = 0;
    f32x4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool do_bias = p.gb && (GEOM == G_UP || t == 0);
    float bsum = 0.f;

    for (size_t m0 = m_begin; m0 < m_end; m0 += kWRows) {
        __syncthreads();
        // stage the input rows: piece = (row, group of 8 channels)
        const int ga = cin / 8;
        for (int q = threadIdx.x; q < kWRows * ga; q += 256) {
            const int row = q % kWRows, cg = q / kWRows;
            const size_t m = m0 + row;
            uint4 raw = {0u, 0u, 0u, 0u};
            if (m < m_end) {
                int z, y, x;
                decompose(m, rows, z, y, x);
                long long v;
                if (GEOM == G_UP) v = (long long)m;
                else v = window_voxel<GEOM>(p.in, z, y, x, t);
                if (v >= 0) {
                    const int ci = cg * 8;
                    const uint16_t* src = ci < p.c0 ? p.x0 + size_t(v) * p.c0 + ci
                                                    : p.x1 + size_t(v) * p.c1 + (ci - p.c0);
                    raw = *reinterpret_cast<const uint4*>(src);
                }
            }
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&raw);
#pragma unroll
            for (int j = 0; j < 8; ++j) la[(cg * 8 + j) * kWPitch + row] = e[j];
        }
        // stage the output-gradient rows
        const int gg = p.cout / 8;
        for (int q = threadIdx.x; q < kWRows * gg; q += 256) {
            const int row = q % kWRows, cg = q / kWRows;
            const size_t m = m0 + row;
            uint4 raw = {0u, 0u, 0u, 0u};
            if (m < m_end) {
                size_t ov = m;
                if (GEOM == G_UP) {
                    int z, y, x;
                    decompose(m, rows, z, y, x);
                    ov = up_voxel(p.out, z, y, x, t);
                }
                raw = *reinterpret_cast<const uint4*>(p.g + ov * size_t(p.cout) + cg * 8);
            }
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&raw);
#pragma unroll
            for (int j = 0; j < 8; ++j) lg[(cg * 8 + j) * kWPitch + row] = e[j];
        }
        __syncthreads();
        const int k0 = wave * 32 + g * 8;
        bf16x8 b[TJ];
#pragma unroll
        for (int j = 0; j < TJ; ++j)
            b[j] = as_bf16x8(*reinterpret_cast<const uint4*>(lg + (j * 16 + r) * kWPitch + k0));
#pragma unroll
        for (int i = 0; i < TI; ++i) {
            const bf16x8 a =
                as_bf16x8(*reinterpret_cast<const uint4*>(la + (i * 16 + r) * kWPitch + k0));
#pragma unroll
            for (int j = 0; j < TJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
        }
        if (do_bias && int(threadIdx.x) < p.cout)
            for (int row = 0; row < kWRows; ++row) bsum += bf2f(lg[threadIdx.x * kWPitch + row]);
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ci = i * 16 + 4 * g + e;
                const int co = j * 16 + r;
                if (ci < p.cin_log && co < p.cout && acc[i][j][e] != 0.f)
                    atomicAdd(p.gw + (size_t(t) * p.cin_log + ci) * p.cout + co, acc[i][j][e]);
            }
    if (do_bias && int(threadIdx.x) < p.cout && bsum != 0.f) atomicAdd(p.gb + threadIdx.x, bsum);
}

// ------------------------------------------------ 3x3x3 weight gradient, LDS tile
// dW[t][ci][co] = sum over output voxels v of X[v + tap t][ci] G[v][co], as
// matrix products with the voxels as the reduction: a lane's 8 reduction
// elements are 8 consecutive voxels along x of one channel, so both operands
// are staged channel-major. A work-group loops over output blocks of 2 x 4 x
// 16 voxels; per block it stages the output gradient G ([co][z][y][x]) and
// the input with its halo as three copies shifted by dx = 0, 1, 2 along x
// ([dx][ci][z][y][x], 16 voxels per row) so that every tap reads 16-byte
// aligned rows; channel pitches are an odd number of 16-byte chunks. Wave w
// accumulates taps w, w+4, ... for all (ci, co) tiles over all its blocks and
// adds them to gw with FP32 atomics at the end; the bias gradient is summed
// from the staged G. One tap's reduction over a block is 4 products of 32
// voxels (two rows of 16 each). Work-group row blockIdx.y takes input
// channels 16 TI blockIdx.y .. 16 TI (blockIdx.y + 1) - 1, so that wide
// layers split their input channels over the grid instead of the LDS.
constexpr int kWBZ = 2, kWBY = 4;  // output block (x: 16)
constexpr int kWRowsX = (kWBZ + 2) * (kWBY + 2);
constexpr int kWXPitch = kWRowsX * 16 + 8;  // per input channel, BF16 (odd 16-byte chunks)
constexpr int kWGPitch = kWBZ * kWBY * 16 + 8;
constexpr int kWTaps = 7;  // taps per wave: ceil(27 / 4)

template <int TI, int TJ>
__host__ __device__ constexpr size_t wtile_lds_bytes()
{
    return (size_t(3) * TI * 16 * kWXPitch + size_t(TJ) * 16 * kWGPitch) * sizeof(uint16_t);
}

template <int TI, int TJ>
__global__ void __launch_bounds__(256) wgrad3_tile_kernel(WgradParams p, int nblocks)
{
    extern __shared__ __align__(16) uint16_t wl[];
    uint16_t* xs = wl;                               // [3][TI*16][kWXPitch]
    uint16_t* gs = wl + 3 * TI * 16 * kWXPitch;      // [TJ*16][kWGPitch]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int ci0 = int(blockIdx.y) * TI * 16;  // first input channel of this row
    const int cin = min(TI * 16, p.c0 + p.c1 - ci0);  // staged here, a multiple of 8
    const int cg = cin / 8, gg = p.cout / 8;
    const int nxt = (p.out.nx + 15) / 16, nyt = (p.out.ny + kWBY - 1) / kWBY;

    // staged channels cin .. TI*16-1 (past the input's last) stay zero
    for (int i = threadIdx.x; i < 3 * (TI * 16 - cin) * kWXPitch; i += 256) {
        const int c = cin + (i / kWXPitch) % (TI * 16 - cin);
        const int d = i / ((TI * 16 - cin) * kWXPitch);
        xs[(d * TI * 16 + c) * kWXPitch + i % kWXPitch] = 0;
    }
    f32x4 acc[kWTaps][TI][TJ];
#pragma unroll
    for (int k = 0; k < kWTaps; ++k)
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[k][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;

    for (int blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const int bx = blk % nxt, by = (blk / nxt) % nyt, bz = blk / (nxt * nyt);
        const int x0 = bx * 16, y0 = by * kWBY, z0 = bz * kWBZ;
        __syncthreads();  // the previous block's reads are done
        // input with halo: piece = (staged voxel, 8 channels) -> the copies it lands in
        for (int q = threadIdx.x; q < kWRowsX * 18 * cg; q += 256) {
            const int c = q % cg, v = q / cg;
            const int lx = v % 18, row = v / 18;
            const int ly = row % (kWBY + 2), lz = row / (kWBY + 2);
            const int ix = x0 + lx - 1, iy = y0 + ly - 1, iz = z0 + lz - 1;
            uint4 raw = {0u, 0u, 0u, 0u};
            if (ix >= 0 && iy >= 0 && iz >= 0 && ix < p.in.nx && iy < p.in.ny && iz < p.in.nz) {
                const size_t gv = (size_t(iz) * p.in.ny + iy) * p.in.nx + ix;
                const int ci = ci0 + c * 8;
                const uint16_t* src =
                    ci < p.c0 ? p.x0 + gv * p.c0 + ci : p.x1 + gv * p.c1 + (ci - p.c0);
                raw = *reinterpret_cast<const uint4*>(src);
            }
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&raw);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int xx = lx - d;  // copy d holds staged x' + d at x'
                if (xx < 0 || xx >= 16) continue;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    xs[(d * TI * 16 + c * 8 + k) * kWXPitch + row * 16 + xx] = e[k];
            }
        }
        // output gradient (zero outside the volume)
        for (int q = threadIdx.x; q < kWBZ * kWBY * 16 * gg; q += 256) {
            const int c = q % gg, v = q / gg;
            const int lx = v % 16, row = v / 16;
            const int ly = row % kWBY, lz = row / kWBY;
            const int ox = x0 + lx, oy = y0 + ly, oz = z0 + lz;
            uint4 raw = {0u, 0u, 0u, 0u};
            if (ox < p.out.nx && oy < p.out.ny && oz < p.out.nz)
                raw = *reinterpret_cast<const uint4*>(
                    p.g + ((size_t(oz) * p.out.ny + oy) * p.out.nx + ox) * p.cout + c * 8);
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&raw);
#pragma unroll
            for (int k = 0; k < 8; ++k) gs[(c * 8 + k) * kWGPitch + row * 16 + lx] = e[k];
        }
        __syncthreads();
        if (p.gb && blockIdx.y == 0 && int(threadIdx.x) < p.cout)
            for (int v = 0; v < kWBZ * kWBY * 16; ++v) bsum += bf2f(gs[threadIdx.x * kWGPitch + v]);
        // four reduction steps of 32 voxels: rows 2kk and 2kk+1, lane group g
        // takes row 2kk + g/2, voxels 8 (g%2) .. 8 (g%2) + 7
#pragma unroll
        for (int kk = 0; kk < kWBZ * kWBY / 2; ++kk) {
            const int rr = 2 * kk + (g >> 1), xo = 8 * (g & 1);
            const int zr = rr / kWBY, yr = rr % kWBY;
            bf16x8 b[TJ];
#pragma unroll
            for (int j = 0; j < TJ; ++j)
                b[j] = as_bf16x8(*reinterpret_cast<const uint4*>(
                    gs + (j * 16 + r) * kWGPitch + rr * 16 + xo));
#pragma unroll
            for (int k = 0; k < kWTaps; ++k) {
                const int t = wave + 4 * k;
                if (t >= 27) break;
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
                const int xrow = (zr + dz) * (kWBY + 2) + (yr + dy);
#pragma unroll
                for (int i = 0; i < TI; ++i) {
                    const bf16x8 a = as_bf16x8(*reinterpret_cast<const uint4*>(
                        xs + (dx * TI * 16 + i * 16 + r) * kWXPitch + xrow * 16 + xo));
#pragma unroll
                    for (int j = 0; j < TJ; ++j)
                        acc[k][i][j] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[k][i][j], 0, 0, 0);
                }
            }
        }
    }
    // lane (r, g) holds dW[ci = 16 i + 4 g + e][co = 16 j + r]
#pragma unroll
    for (int k = 0; k < kWTaps; ++k) {
        const int t = wave + 4 * k;
        if (t >= 27) break;
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ci = ci0 + i * 16 + 4 * g + e, co = j * 16 + r;
                    if (ci < p.cin_log && acc[k][i][j][e] != 0.f)
                        atomicAdd(p.gw + (size_t(t) * p.cin_log + ci) * p.cout + co,
                                  acc[k][i][j][e]);
                }
    }
    if (p.gb && blockIdx.y == 0 && int(threadIdx.x) < p.cout && bsum != 0.f)
        atomicAdd(p.gb + threadIdx.x, bsum);
}

// ------------------------------------------------------------------- packing
__global__ void __launch_bounds__(256)
pack_kernel(const float* __restrict__ w, int taps, int cin_log, int cin, int cout, int mode, int K,
            int N, int kblocks, size_t total, uint16_t* __restrict__ packed)
{
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int i = int(idx & 7);
    const int lane = int((idx >> 3) & 63);
    const size_t blk = idx >> 9;
    const int kb = int(blk % size_t(kblocks));
    const int nt = int(blk / size_t(kblocks));
    const int k = kb * 32 + (lane >> 4) * 8 + i;
    const int n = nt * 16 + (lane & 15);
    float v = 0.f;
    if (k < K && n < N) {
        int t = 0, ci = 0, co = 0;
        switch (mode) {
        case PACK_FWD: t = k / cin; ci = k - t * cin; co = n; break;
        case PACK_FWD_UP: ci = k; t = n / cout; co = n - t * cout; break;
        case PACK_BWD_FLIP: t = k / cout; co = k - t * cout; ci = n; t = taps - 1 - t; break;
        case PACK_BWD: t = k / cout; co = k - t * cout; ci = n; break;
        default: co = k; t = n / cin; ci = n - t * cin; break;  // PACK_BWD_UP
        }
        if (ci < cin_log) v = w[(size_t(t) * cin_log + ci) * cout + co];
    }
    packed[idx] = f2bf(v);
}

// --------------------------------------------------------------- elementwise
__global__ void __launch_bounds__(256)
pack_input_kernel(const float* __restrict__ dose, const float* __restrict__ sigma,
                  const float* __restrict__ rho, float inv_dmax, size_t n, uint16_t* __restrict__ x)
{
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint4 o;
    o.x = uint32_t(f2bf(dose[v] * inv_dmax)) | (uint32_t(f2bf(sigma[v] * inv_dmax)) << 16);
    o.y = uint32_t(f2bf(rho[v] * 0.5f));
    o.z = 0u;
    o.w = 0u;
    reinterpret_cast<uint4*>(x)[v] = o;
}

__global__ void __launch_bounds__(256)
head_fwd_kernel(const uint16_t* __restrict__ dec, const float* __restrict__ wh,
                const float* __restrict__ bh, const float* __restrict__ dose, float inv_dmax,
                size_t n, float* __restrict__ y, float* __restrict__ out)
{
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint4* d = reinterpret_cast<const uint4*>(dec + v * 16);
    float s = bh[0];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint4 q = d[h];
        const uint32_t wds[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s += bf2f(uint16_t(wds[j] & 0xffffu)) * wh[h * 8 + 2 * j];
            s += bf2f(uint16_t(wds[j] >> 16)) * wh[h * 8 + 2 * j + 1];
        }
    }
    const float yn = dose[v] * inv_dmax + s;
    if (y) y[v] = yn;
    if (out) out[v] = yn / inv_dmax;
}

__device__ __forceinline__ float block_sum(float x, float* s_w)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    float t = 0.f;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) t += s_w[w];
    return t;
}

__global__ void __launch_bounds__(256)
max_kernel(const float* __restrict__ a, float scale, size_t n, float* __restrict__ out)
{
    __shared__ float s_m[4];
    float m = 0.f;
    for (size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += size_t(gridDim.x) * blockDim.x)
        m = fmaxf(m, a[v] * scale);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    // one atomic per work-group (non-negative floats order as their bit patterns)
    if (threadIdx.x == 0) {
        for (int w = 1; w < int(blockDim.x >> 6); ++w) m = fmaxf(m, s_m[w]);
        if (m > 0.f) atomicMax(reinterpret_cast<unsigned int*>(out), __float_as_uint(m));
    }
}

__global__ void __launch_bounds__(256)
loss_sum_kernel(const float* __restrict__ y, const float* __restrict__ target, float inv_dmax,
                size_t n, float* __restrict__ sums)
{
    __shared__ float s_w[4];
    const float thr = 0.1f * sums[0];
    float sw = 0.f, sl = 0.f;
    for (size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += size_t(gridDim.x) * blockDim.x) {
        const float t = target[v] * inv_dmax;
        const float w = t > thr ? 1.f : 0.1f;
        const float r = y[v] - t;
        sw += w;
        sl += w * r * r;
    }
    sw = block_sum(sw, s_w);
    sl = block_sum(sl, s_w);
    if (threadIdx.x == 0) {
        atomicAdd(sums + 1, sw);
        atomicAdd(sums + 2, sl);
    }
}

__global__ void __launch_bounds__(256)
loss_grad_kernel(const float* __restrict__ y, const float* __restrict__ target, float inv_dmax,
                 size_t n, const float* __restrict__ sums, float* __restrict__ gy)
{
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const float t = target[v] * inv_dmax;
    const float w = t > 0.1f * sums[0] ? 1.f : 0.1f;
    gy[v] = 2.f * w * (y[v] - t) / sums[1];
}

// Four threads per voxel, each with 4 of the 16 channels: the 8-byte read of
// dec and the 16-byte write of gdec of consecutive threads are contiguous.
__global__ void __launch_bounds__(256)
head_bwd_kernel(const uint16_t* __restrict__ dec, const float* __restrict__ gy,
                const float* __restrict__ wh, size_t n, float* __restrict__ gwh,
                float* __restrict__ gbh, float* __restrict__ gdec)
{
    __shared__ float s_c[4][16];
    __shared__ float s_b[4];
    const int q = threadIdx.x & 3;  // channels 4q .. 4q+3
    const float4 w = float4{wh[4 * q], wh[4 * q + 1], wh[4 * q + 2], wh[4 * q + 3]};
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, sb = 0.f;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < 4 * n;
         i += size_t(gridDim.x) * blockDim.x) {
        const size_t v = i >> 2;
        const float gv = gy[v];
        if (q == 0) sb += gv;
        const uint2 d = reinterpret_cast<const uint2*>(dec)[i];
        a0 += gv * bf2f(uint16_t(d.x & 0xffffu));
        a1 += gv * bf2f(uint16_t(d.x >> 16));
        a2 += gv * bf2f(uint16_t(d.y & 0xffffu));
        a3 += gv * bf2f(uint16_t(d.y >> 16));
        reinterpret_cast<float4*>(gdec)[i] = float4{gv * w.x, gv * w.y, gv * w.z, gv * w.w};
    }
    // sum over the lanes of the same channel quarter, then over the waves
#pragma unroll
    for (int off = 4; off < 64; off <<= 1) {
        a0 += __shfl_xor(a0, off);
        a1 += __shfl_xor(a1, off);
        a2 += __shfl_xor(a2, off);
        a3 += __shfl_xor(a3, off);
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) sb += __shfl_xor(sb, off);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) < 4) {
        s_c[wv][4 * q + 0] = a0;
        s_c[wv][4 * q + 1] = a1;
        s_c[wv][4 * q + 2] = a2;
        s_c[wv][4 * q + 3] = a3;
    }
    if ((threadIdx.x & 63) == 0) s_b[wv] = sb;
    __syncthreads();
    if (threadIdx.x < 16) {
        float t = 0.f;
        for (int k = 0; k < int(blockDim.x >> 6); ++k) t += s_c[k][threadIdx.x];
        atomicAdd(gwh + threadIdx.x, t);
    } else if (threadIdx.x == 16) {
        float t = 0.f;
        for (int k = 0; k < int(blockDim.x >> 6); ++k) t += s_b[k];
        atomicAdd(gbh, t);
    }
}

// Eight elements per thread (n is a multiple of 8: channels come in eights).
__global__ void __launch_bounds__(256)
relu_bwd_kernel(const float* __restrict__ g, const uint16_t* __restrict__ act, size_t n8,
                uint16_t* __restrict__ out)
{
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const uint4 a = reinterpret_cast<const uint4*>(act)[i];
    const float4 g0 = reinterpret_cast<const float4*>(g)[2 * i];
    const float4 g1 = reinterpret_cast<const float4*>(g)[2 * i + 1];
    const uint32_t aw[4] = {a.x, a.y, a.z, a.w};
    const float gf[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t r = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t b = (aw[k] >> (16 * h)) & 0xffffu;
            const uint32_t y = (b & 0x7fffu) != 0u && !(b & 0x8000u) ? f2bf(gf[2 * k + h]) : 0u;
            r |= y << (16 * h);
        }
        o[k] = r;
    }
    reinterpret_cast<uint4*>(out)[i] = uint4{o[0], o[1], o[2], o[3]};
}

__global__ void __launch_bounds__(256)
adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
            const float* __restrict__ g, size_t n, float lr, float b1, float b2, float eps,
            float bc1, float bc2)
{
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void __launch_bounds__(256)
f32_to_bf16_kernel(const float* __restrict__ in, size_t n, uint16_t* __restrict__ out)
{
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(in[i]);
}

__global__ void __launch_bounds__(256)
bf16_to_f32_kernel(const uint16_t* __restrict__ in, size_t n, float* __restrict__ out)
{
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = bf2f(in[i]);
}

__device__ __forceinline__ double block_sum_d(double x, double* s_w)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) t += s_w[w];
    return t;
}

__global__ void __launch_bounds__(256)
dn_error_kernel(const float* __restrict__ dn, const float* __restrict__ lo,
                const float* __restrict__ sigma, size_t n, const float* __restrict__ lmax,
                double* __restrict__ acc)
{
    __shared__ double s_w[4];
    const float thr = 0.1f * lmax[0];
    double c = 0.0, d2 = 0.0, s2 = 0.0;
    for (size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += size_t(gridDim.x) * blockDim.x) {
        if (lo[v] > thr) {
            const double d = double(dn[v]) - double(lo[v]);
            c += 1.0;
            d2 += d * d;
            s2 += double(sigma[v]) * double(sigma[v]);
        }
    }
    c = block_sum_d(c, s_w);
    d2 = block_sum_d(d2, s_w);
    s2 = block_sum_d(s2, s_w);
    if (threadIdx.x == 0) {
        atomicAdd(acc + 1, c);
        atomicAdd(acc + 2, d2);
        atomicAdd(acc + 3, s2);
    }
}

__global__ void copy_max_kernel(const float* m, double* acc)
{
    if (threadIdx.x == 0) acc[0] = double(m[0]);
}

unsigned grid_for(size_t n) { return unsigned((n + 255) / 256); }
// reductions that end in one atomic per work-group on a single address
unsigned grid_reduce(size_t n)
{
    const size_t g = (n + 255) / 256;
    return unsigned(g < 512 ? (g ? g : 1) : 512);
}
unsigned grid_strided(size_t n)
{
    const size_t g = (n + 255) / 256;
    return unsigned(g < 2048 ? (g ? g : 1) : 2048);
}

template <int GEOM, int NT>
int conv_launch(const ConvParams& p, dim3 grid, hipStream_t s)
{
    hipLaunchKernelGGL((conv_kernel<GEOM, NT>), grid, dim3(256), 0, s, p);
    return status();
}

// Dynamic LDS above the default 64 KB needs the kernel's limit raised on the
// current device (a host call, made before each such launch).
int allow_lds(const void* fn, size_t bytes)
{
    if (bytes <= 65536) return 0;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) ==
                   hipSuccess
               ? 0
               : -1;
}

// Largest LDS block a tile kernel takes (96 channels: one work-group per CU).
constexpr size_t kTileLdsMax = 96 * 1024;

template <int NT, int CIN>
int tile_launch(const ConvParams& p, int tiles, hipStream_t s)
{
    using S = TileShape<CIN>;
    static_assert(S::lds <= kTileLdsMax, "staged block within the LDS budget");
    if (allow_lds((const void*)conv3_tile_kernel<NT, CIN>, S::lds)) return -1;
    const unsigned nxt = unsigned((p.out.nx + kTileX - 1) / kTileX);
    const unsigned nyt = unsigned((p.out.ny + S::BY - 1) / S::BY);
    const unsigned nzt = unsigned((p.out.nz + S::BZ - 1) / S::BZ);
    const dim3 grid{nxt * nyt, nzt, unsigned(tiles / NT)};
    hipLaunchKernelGGL((conv3_tile_kernel<NT, CIN>), grid, dim3(256), S::lds, s, p);
    return status();
}

template <int CIN>
int tile_cin(const ConvParams& p, int nt, int tiles, hipStream_t s)
{
    switch (nt) {
    case 1: return tile_launch<1, CIN>(p, tiles, s);
    case 2: return tile_launch<2, CIN>(p, tiles, s);
    case 3: return tile_launch<3, CIN>(p, tiles, s);
    case 4: return tile_launch<4, CIN>(p, tiles, s);
    default: return -1;
    }
}

// The LDS tile path of a 3x3x3 convolution for the channel counts it is
// built for (the network's); the gather kernel runs for others.
bool conv3_tiles(int cin)
{
    return cin == 8 || cin == 16 || cin == 32 || cin == 48 || cin == 64 || cin == 96;
}

// Column tiles per work-group: as many as divide the columns while the grid
// still has two work-groups per CU; fewer (each restages its block) when the
// volume is small.
int tile_columns(int tiles, size_t blocks)
{
    int nt = tiles % 4 == 0 ? 4 : tiles % 3 == 0 ? 3 : tiles % 2 == 0 ? 2 : 1;
    while (nt > 1 && blocks * size_t(tiles / nt) < 512) {
        int next = nt - 1;
        while (next > 1 && tiles % next) --next;
        nt = next;
    }
    return nt;
}

int conv3_tiled(const ConvParams& p, int tiles, hipStream_t s)
{
    const int cin = p.c0 + p.c1;
    const int bz = cin <= 48 ? 4 : 2;
    const size_t blocks = size_t((p.out.nx + kTileX - 1) / kTileX) * ((p.out.ny + 3) / 4) *
                          ((p.out.nz + bz - 1) / bz);
    const int nt = tile_columns(tiles, blocks);
    switch (cin) {
    case 8: return tile_cin<8>(p, nt, tiles, s);
    case 16: return tile_cin<16>(p, nt, tiles, s);
    case 32: return tile_cin<32>(p, nt, tiles, s);
    case 48: return tile_cin<48>(p, nt, tiles, s);
    case 64: return tile_cin<64>(p, nt, tiles, s);
    case 96: return tile_cin<96>(p, nt, tiles, s);
    default: return -1;
    }
}

template <int GEOM>
int conv_geom(const ConvParams& p, int nt, dim3 grid, hipStream_t s)
{
    switch (nt) {
    case 1: return conv_launch<GEOM, 1>(p, grid, s);
    case 2: return conv_launch<GEOM, 2>(p, grid, s);
    case 3: return conv_launch<GEOM, 3>(p, grid, s);
    case 4: return conv_launch<GEOM, 4>(p, grid, s);
    default: return -1;
    }
}

template <int GEOM, int TI, int TJ>
int wgrad_launch(const WgradParams& p, dim3 grid, hipStream_t s)
{
    const size_t lds = size_t(TI + TJ) * 16 * kWPitch * sizeof(uint16_t);
    hipLaunchKernelGGL((wgrad_kernel<GEOM, TI, TJ>), grid, dim3(256), lds, s, p);
    return status();
}

template <int TI, int TJ>
int wgrad_tile_launch(const WgradParams& p, int ci_rows, int cus, hipStream_t s)
{
    constexpr size_t lds = wtile_lds_bytes<TI, TJ>();
    if (allow_lds((const void*)wgrad3_tile_kernel<TI, TJ>, lds)) return -1;
    const int nblocks = ((p.out.nx + 15) / 16) * ((p.out.ny + kWBY - 1) / kWBY) *
                        ((p.out.nz + kWBZ - 1) / kWBZ);
    if (nblocks == 0) return 0;
    int grid = 2 * cus;
    if (grid > nblocks) grid = nblocks;
    hipLaunchKernelGGL((wgrad3_tile_kernel<TI, TJ>), dim3(unsigned(grid), unsigned(ci_rows)),
                       dim3(256), lds, s, p, nblocks);
    return status();
}

// the (input tiles, output tiles) shapes of the network's layers
template <int GEOM>
int wgrad_geom(const WgradParams& p, int ti, int tj, dim3 grid, hipStream_t s)
{
#define OMC_WG(a, b) \
    if (ti == a && tj == b) return wgrad_launch<GEOM, a, b>(p, grid, s);
    OMC_WG(1, 1) OMC_WG(2, 2) OMC_WG(3, 3) OMC_WG(4, 4) OMC_WG(2, 1) OMC_WG(4, 2)
    OMC_WG(6, 3) OMC_WG(1, 2) OMC_WG(2, 3) OMC_WG(3, 4) OMC_WG(4, 3) OMC_WG(3, 2)
#undef OMC_WG
    return -1;
}

}  // namespace

int pack_kblocks(int K) { return (K + 31) / 32; }
int pack_ntiles(int N) { return (N + 15) / 16; }
size_t pack_elems(int K, int N) { return size_t(pack_kblocks(K)) * pack_ntiles(N) * 64 * 8; }

int launch_pack(const float* w, int taps, int cin_log, int cin, int cout, int mode,
                uint16_t* packed, void* stream)
{
    int K, N;
    switch (mode) {
    case PACK_FWD: K = taps * cin; N = cout; break;
    case PACK_FWD_UP: K = cin; N = taps * cout; break;
    case PACK_BWD_FLIP:
    case PACK_BWD: K = taps * cout; N = cin; break;
    case PACK_BWD_UP: K = cout; N = taps * cin; break;
    default: return -1;
    }
    const size_t total = pack_elems(K, N);
    hipLaunchKernelGGL(pack_kernel, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, w,
                       taps, cin_log, cin, cout, mode, K, N, pack_kblocks(K), total, packed);
    return status();
}

int launch_conv(int geometry, const uint16_t* x0, int c0, const uint16_t* x1, int c1, Dims in,
                Dims out, const uint16_t* packed, int K, int N, const ConvOut& o, void* stream)
{
    if (c0 % 8 || c1 % 8 || N % 16 || (geometry == G_UP && N % 128)) return -1;
    ConvParams p;
    p.x0 = x0;
    p.x1 = x1;
    p.c0 = c0;
    p.c1 = c1;
    p.in = in;
    p.out = out;
    p.packed = packed;
    p.K = K;
    p.N = N;
    p.kblocks = pack_kblocks(K);
    p.M = geometry == G_UP ? in.vox() : out.vox();
    p.o = o;
    const int tiles = N / 16;
    const int nt = tiles % 4 == 0 ? 4 : tiles % 3 == 0 ? 3 : tiles % 2 == 0 ? 2 : 1;
    const dim3 grid{unsigned((p.M + 255) / 256), unsigned(tiles / nt), 1u};
    hipStream_t s = (hipStream_t)stream;
    switch (geometry) {
    case G_CONV3:
        if (in.nz == out.nz && in.ny == out.ny && in.nx == out.nx && conv3_tiles(c0 + c1))
            return conv3_tiled(p, tiles, s);
        return conv_geom<G_CONV3>(p, nt, grid, s);
    case G_DOWN: return conv_geom<G_DOWN>(p, nt, grid, s);
    case G_UP: return conv_geom<G_UP>(p, nt, grid, s);
    default: return -1;
    }
}

int launch_conv_wgrad(int geometry, const uint16_t* x0, int c0, const uint16_t* x1, int c1,
                      Dims in, Dims out, const uint16_t* g, int cout, int cin_log, float* gw,
                      float* gb, void* stream)
{
    if (c0 % 8 || c1 % 8 || cout % 16) return -1;
    WgradParams p;
    p.x0 = x0;
    p.x1 = x1;
    p.c0 = c0;
    p.c1 = c1;
    p.in = in;
    p.out = out;
    p.g = g;
    p.cout = cout;
    p.cin_log = cin_log;
    p.gw = gw;
    p.gb = gb;
    p.M = geometry == G_UP ? in.vox() : out.vox();
    const int taps = geometry == G_CONV3 ? 27 : 8;
    // about 2048 work-groups over taps x row ranges, whole 128-row steps each
    size_t blocks_x = (2048 + taps - 1) / taps;
    const size_t steps = (p.M + kWRows - 1) / kWRows;
    if (blocks_x > steps) blocks_x = steps;
    const size_t steps_per = (steps + blocks_x - 1) / blocks_x;
    p.rows_per_block = steps_per * kWRows;
    blocks_x = (p.M + p.rows_per_block - 1) / p.rows_per_block;
    const dim3 grid{unsigned(blocks_x), unsigned(taps), 1u};
    const int ti = (c0 + c1 + 15) / 16, tj = cout / 16;
    hipStream_t s = (hipStream_t)stream;
    if (geometry == G_CONV3 && in.nz == out.nz && in.ny == out.ny && in.nx == out.nx) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return -1;
        // the staged-block kernel for the network's shapes: (input tiles per
        // work-group, output tiles), input tiles beyond split over grid rows
        if (tj == 1 && ti <= 2) return ti == 1 ? wgrad_tile_launch<1, 1>(p, 1, cus, s)
                                               : wgrad_tile_launch<2, 1>(p, 1, cus, s);
        if (tj == 2 && ti % 2 == 0) return wgrad_tile_launch<2, 2>(p, ti / 2, cus, s);
        if (tj == 3 && ti % 2 == 0) return wgrad_tile_launch<2, 3>(p, ti / 2, cus, s);
        if (tj == 3) return wgrad_tile_launch<1, 3>(p, ti, cus, s);
        if (tj == 4) return wgrad_tile_launch<1, 4>(p, ti, cus, s);
    }
    switch (geometry) {
    case G_CONV3: return wgrad_geom<G_CONV3>(p, ti, tj, grid, s);
    case G_DOWN: return wgrad_geom<G_DOWN>(p, ti, tj, grid, s);
    case G_UP: return wgrad_geom<G_UP>(p, ti, tj, grid, s);
    default: return -1;
    }
}

int launch_pack_input(const float* dose, const float* sigma, const float* rho, float inv_dmax,
                      size_t n, uint16_t* x, void* stream)
{
    hipLaunchKernelGGL(pack_input_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                       dose, sigma, rho, inv_dmax, n, x);
    return status();
}

int launch_head_fwd(const uint16_t* dec, const float* wh, const float* bh, const float* dose,
                    float inv_dmax, size_t n, float* y, float* out, void* stream)
{
    hipLaunchKernelGGL(head_fwd_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, dec,
                       wh, bh, dose, inv_dmax, n, y, out);
    return status();
}

int launch_loss(const float* y, const float* target, float inv_dmax, size_t n, float* sums,
                float* gy, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(max_kernel, dim3(grid_reduce(n)), dim3(256), 0, s, target, inv_dmax, n,
                       sums);
    hipLaunchKernelGGL(loss_sum_kernel, dim3(grid_strided(n)), dim3(256), 0, s, y, target,
                       inv_dmax, n, sums);
    if (gy)
        hipLaunchKernelGGL(loss_grad_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, target,
                           inv_dmax, n, sums, gy);
    return status();
}

int launch_head_bwd(const uint16_t* dec, const float* gy, const float* wh, size_t n, float* gwh,
                    float* gbh, float* gdec, void* stream)
{
    hipLaunchKernelGGL(head_bwd_kernel, dim3(grid_strided(4 * n)), dim3(256), 0,
                       (hipStream_t)stream, dec, gy, wh, n, gwh, gbh, gdec);
    return status();
}

int launch_relu_bwd(const float* g, const uint16_t* act, size_t n, uint16_t* out, void* stream)
{
    if (n % 8) return -1;
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(grid_for(n / 8)), dim3(256), 0, (hipStream_t)stream,
                       g, act, n / 8, out);
    return status();
}

int launch_adam(float* p, float* m, float* v, const float* g, size_t n, float lr, float b1,
                float b2, float eps, float bc1, float bc2, void* stream)
{
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, p, m, v,
                       g, n, lr, b1, b2, eps, bc1, bc2);
    return status();
}

int launch_f32_to_bf16(const float* in, size_t n, uint16_t* out, void* stream)
{
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                       in, n, out);
    return status();
}

int launch_bf16_to_f32(const uint16_t* in, size_t n, float* out, void* stream)
{
    hipLaunchKernelGGL(bf16_to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                       in, n, out);
    return status();
}

int launch_dn_error(const float* dn, const float* lo, const float* sigma, size_t n, double* acc,
                    void* stream)
{
    // acc[4] (as float) holds the running maximum of lo
    hipStream_t s = (hipStream_t)stream;
    float* lmax = reinterpret_cast<float*>(acc + 4);
    hipLaunchKernelGGL(max_kernel, dim3(grid_reduce(n)), dim3(256), 0, s, lo, 1.0f, n, lmax);
    hipLaunchKernelGGL(dn_error_kernel, dim3(grid_strided(n)), dim3(256), 0, s, dn, lo, sigma, n,
                       lmax, acc);
    hipLaunchKernelGGL(copy_max_kernel, dim3(1), dim3(64), 0, s, lmax, acc);
    return status();
}

}  // namespace dn
