// Initial state and the one-lattice half-sweep kernels for gfx950; the
// per-thread update is in sweep_device.h.
#include <algorithm>

#include "internal.h"
#include "sweep_device.h"

namespace mcl {
namespace {


// ---------------------------------------------------------------------------
// Initial state.  One thread per 32-bit word (8 cells) of one plane.
// ---------------------------------------------------------------------------
// Word g of the two planes (plane-major, then row, then word).
__device__ __forceinline__ uint32_t init_word(int64_t g, int64_t L, int64_t W, int model, int init_state,
                                              uint32_t k0, uint32_t k1)
{
    const int color = (int)(g / (L * W));
    const int64_t rem = g - (int64_t)color * L * W;
    const int64_t y = rem / W;
    const int64_t wd = rem - y * W;
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        int s;
        if (init_state == 1) {
            s = 1;
        } else if (init_state == 2) {
            s = -1;
        } else if (init_state == 3) {
            s = 0;
        } else {
            const int64_t i = wd * 8 + j;
            const int64_t x = 2 * i + ((y + color) & 1);
            const uint64_t n = (uint64_t)(y * L + x);
            const uint64_t blk = n >> 2;
            const Philox4 o = philox4x32_10(dev::lo32(blk), dev::hi32(blk), 0u, 4u, k0, k1);
            const uint32_t sel = (uint32_t)(n & 3);
            const uint32_t w = sel == 0 ? o.v0 : sel == 1 ? o.v1 : sel == 2 ? o.v2 : o.v3;
            if (model == 0)
                s = (w < 0x80000000u) ? 1 : -1;
            else
                s = (int)(((uint64_t)w * 3u) >> 32) - 1;
        }
        word |= (uint32_t)(s + 1) << (4 * j);
    }
    return word;
}

__global__ __launch_bounds__(256) void init_kernel(uint32_t* __restrict__ planes, int64_t L, int64_t W,
                                                   int model, int init_state, uint32_t k0, uint32_t k1)
{
    const int64_t total = 2 * L * W;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x)
        planes[g] = init_word(g, L, W, model, init_state, k0, k1);
}

// The sweep index of a launch is t, plus the device word *tbase when tbase
// is given (a captured graph replays the same launches at any starting t).
template <int MODEL, bool HI0, int COLOR>
__global__ __launch_bounds__(256) void half_sweep_kernel(uint32_t* __restrict__ own, const uint32_t* __restrict__ oth,
                                                         uint32_t L, uint32_t rows, uint32_t t,
                                                         const uint32_t* __restrict__ tbase, uint32_t k0,
                                                         uint32_t k1, uint32_t T4, uint32_t T8, BCTable tbl)
{
    __shared__ dev::BCLds s_tab;
    if (tbase) t += *tbase;
    if (MODEL == 1) dev::load_bc_table(s_tab, tbl);
    const uint32_t Q = L >> 6;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t q = g % Q;
    const uint32_t band = g / Q;
    const uint32_t y0 = band * rows;
    if (y0 >= L) return;
    // a row of a whole number of waves: the wave's row terms are scalar
    if ((Q & 63u) == 0u) {
        dev::band_update_wave<MODEL, HI0, COLOR>(own, oth, L, rows, q, y0, t, k0, k1, T4, T8, s_tab.e);
        return;
    }
    // blocks of the band: accept draws of in-colour cells y0 L/2 + 32 q .. (y0 + rows - 1) L/2 + 32 q + 31
    uint32_t hu;
    const int hm = dev::counter_mode(HI0, ((uint64_t)y0 * (L >> 1) + 32u * q) >> 2,
                                     ((uint64_t)(y0 + rows - 1) * (L >> 1) + 32u * q + 31u) >> 2, hu);
    if (hm == 0)
        dev::band_update<MODEL, 0, COLOR>(own, oth, L, rows, q, y0, t, k0, k1, 0u, T4, T8, s_tab.e);
    else if (hm == 1)
        dev::band_update<MODEL, 1, COLOR>(own, oth, L, rows, q, y0, t, k0, k1, hu, T4, T8, s_tab.e);
    else
        dev::band_update<MODEL, 2, COLOR>(own, oth, L, rows, q, y0, t, k0, k1, 0u, T4, T8, s_tab.e);
}

// Initial state of the 1-bit layout: one thread per word (32 cells) of one plane.
__device__ __forceinline__ uint32_t init1_word(int64_t g, int64_t L, int64_t W, int init_state, uint32_t k0,
                                               uint32_t k1)
{
    const int color = (int)(g / (L * W));
    const int64_t rem = g - (int64_t)color * L * W;
    const int64_t y = rem / W;
    const int64_t wd = rem - y * W;
    if (init_state == 1) return 0xFFFFFFFFu;
    if (init_state == 2) return 0u;
    uint32_t word = 0;
    for (int j = 0; j < 32; ++j) {
        const int64_t x = 2 * (wd * 32 + j) + ((y + color) & 1);
        const uint64_t n = (uint64_t)(y * L + x);
        const Philox4 o = philox4x32_10(dev::lo32(n >> 2), dev::hi32(n >> 2), 0u, 4u, k0, k1);
        word |= (philox_word(o, (int)(n & 3)) < 0x80000000u ? 1u : 0u) << j;
    }
    return word;
}

__global__ __launch_bounds__(256) void init1_kernel(uint32_t* __restrict__ planes, int64_t L, int64_t W,
                                                    int init_state, uint32_t k0, uint32_t k1)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < 2 * L * W;
         g += (int64_t)gridDim.x * blockDim.x)
        planes[g] = init1_word(g, L, W, init_state, k0, k1);
}

// Bucket table of the 1-bit mode, one thread per bucket (the entry is
// lut_bucket_addend of sweep_device.h).
__global__ __launch_bounds__(256) void lut_bucket_kernel(LutTable tab, uint2* __restrict__ out)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= (uint32_t)dev::kLutBuckets) return;
    const uint64_t A = dev::lut_bucket_addend(tab.T, tab.kmax, b);
    out[b] = make_uint2((uint32_t)A, (uint32_t)(A >> 32));
}

template <bool HI0, int COLOR>
__global__ __launch_bounds__(512) void lut_half_kernel(uint32_t* __restrict__ own, const uint32_t* __restrict__ oth,
                                                       uint32_t L, uint32_t rows, uint32_t t,
                                                       const uint32_t* __restrict__ tbase, uint32_t k0, uint32_t k1,
                                                       LutTable tab, const uint2* __restrict__ buckets)
{
    if (tbase) t += *tbase;
    __shared__ uint32_t s_lut[16];
    __shared__ uint2 s_b[dev::kLutBuckets];
    if (threadIdx.x < 16) s_lut[threadIdx.x] = tab.T[threadIdx.x];
    {
        const uint4* src = reinterpret_cast<const uint4*>(buckets);
        uint4* dst = reinterpret_cast<uint4*>(s_b);
        for (uint32_t i = threadIdx.x; i < (uint32_t)dev::kLutBuckets / 2; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    const uint32_t Q = L >> 8;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t q = g % Q;
    const uint32_t y0 = (g / Q) * rows;
    if (y0 >= L) return;
    // blocks of the band: groups of 16 in-colour cells, y0 L/2 + 128 q .. (y0 + rows - 1) L/2 + 128 q + 127
    uint32_t hu;
    const int hm = dev::counter_mode(HI0, ((uint64_t)y0 * (L >> 1) + 128u * q) >> 4,
                                     ((uint64_t)(y0 + rows - 1) * (L >> 1) + 128u * q + 127u) >> 4, hu);
    if (hm == 0)
        dev::band_update_lut<0, COLOR>(own, oth, L, rows, q, y0, t, k0, k1, 0u, s_b, s_lut, tab.T[8], tab.kmax);
    else if (hm == 1)
        dev::band_update_lut<1, COLOR>(own, oth, L, rows, q, y0, t, k0, k1, hu, s_b, s_lut, tab.T[8], tab.kmax);
    else
        dev::band_update_lut<2, COLOR>(own, oth, L, rows, q, y0, t, k0, k1, 0u, s_b, s_lut, tab.T[8], tab.kmax);
}

// Band height (rows per thread, even, dividing L): 32 amortises the two
// halo rows of the other plane (1/16 extra reads); smaller lattices take
// shorter bands until a launch has 2^20 threads (16 waves per SIMD) --
// Q vectors per row, L rows.  Measured against targets of 2^17 to 2^22
// threads: 2^20 is the best or within 1% at every L, and up to 26% faster
// than 2^17 at L = 2^13..2^15 (other waves hide the latency of each
// thread's chain of row steps); L >= 2^16 (4-bit) keeps 32 rows either way.
int64_t band_rows(int64_t Q, int64_t L)
{
    int64_t rows = 32;
    while (rows > 2 && Q * (L / rows) < (int64_t(1) << 20)) rows >>= 1;
    return rows;
}

}  // namespace

// One launch covers at most 2^32 work-items per dimension: the init
// kernels stride over the planes with a grid of at most 2^20 workgroups.
constexpr int64_t kMaxInitBlocks = int64_t(1) << 20;

hipError_t launch_init(const Geom& g, int model, int init_state, uint64_t seed, hipStream_t s)
{
    const int64_t total = 2 * g.L * g.W;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, kMaxInitBlocks);
    hipLaunchKernelGGL(init_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, g.plane0, g.L, g.W, model,
                       init_state, (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

template <int MODEL, bool HI0>
static void launch_model(dim3 grid, hipStream_t s, uint32_t* own, const uint32_t* oth, uint32_t L, uint32_t R, int c,
                         uint32_t t, const uint32_t* tbase, uint32_t k0, uint32_t k1, uint32_t T4, uint32_t T8,
                         const BCTable& tbl)
{
    if (c == 0)
        hipLaunchKernelGGL((half_sweep_kernel<MODEL, HI0, 0>), grid, dim3(256), 0, s, own, oth, L, R, t, tbase, k0,
                           k1, T4, T8, tbl);
    else
        hipLaunchKernelGGL((half_sweep_kernel<MODEL, HI0, 1>), grid, dim3(256), 0, s, own, oth, L, R, t, tbase, k0,
                           k1, T4, T8, tbl);
}

static hipError_t launch_half(const Geom& g, const HalfSweepArgs& a, hipStream_t s, int model)
{
    const int64_t rows = band_rows(g.Q, g.L);
    const int64_t threads = g.Q * (g.L / rows);
    const int64_t blocks = (threads + 255) / 256;
    BCTable tbl{};
    if (a.bc) tbl = *a.bc;
    uint32_t* own = g.plane(a.color);
    const uint32_t* oth = g.plane(1 - a.color);
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    // block indices fit 32 bits while L^2 / 8 <= 2^32
    const bool hi0 = (g.L * g.L / 8) <= (int64_t(1) << 32);
    const uint32_t L = (uint32_t)g.L, R = (uint32_t)rows;
    const dim3 grid((uint32_t)blocks);
    if (model == 0) {
        if (hi0) launch_model<0, true>(grid, s, own, oth, L, R, a.color, a.t, a.tbase, k0, k1, a.T4, a.T8, tbl);
        else launch_model<0, false>(grid, s, own, oth, L, R, a.color, a.t, a.tbase, k0, k1, a.T4, a.T8, tbl);
    } else {
        if (hi0) launch_model<1, true>(grid, s, own, oth, L, R, a.color, a.t, a.tbase, k0, k1, a.T4, a.T8, tbl);
        else launch_model<1, false>(grid, s, own, oth, L, R, a.color, a.t, a.tbase, k0, k1, a.T4, a.T8, tbl);
    }
    return hipGetLastError();
}

hipError_t launch_init1(const Geom& g, int init_state, uint64_t seed, hipStream_t s)
{
    const int64_t total = 2 * g.L * g.W;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, kMaxInitBlocks);
    hipLaunchKernelGGL(init1_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, g.plane0, g.L, g.W,
                       init_state, (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_lut_buckets(const LutTable& tab, void* buckets, hipStream_t s)
{
    hipLaunchKernelGGL(lut_bucket_kernel, dim3(dev::kLutBuckets / 256), dim3(256), 0, s, tab,
                       reinterpret_cast<uint2*>(buckets));
    return hipGetLastError();
}

hipError_t launch_lut_half(const Geom& g, int color, uint32_t t, const uint32_t* tbase, uint64_t seed,
                           const LutTable& tab, const void* buckets, hipStream_t s)
{
    const uint2* bk = reinterpret_cast<const uint2*>(buckets);
    const int64_t rows = band_rows(g.Q, g.L);
    const int64_t threads = g.Q * (g.L / rows);
    // 512-thread workgroups: each copies the 32 KiB bucket table into LDS
    // once, so larger groups copy it fewer times per update (measured 0.4-3.6%
    // faster than 256 threads at L = 2^13..2^17; 1024 threads lose occupancy)
    const dim3 grid((uint32_t)((threads + 511) / 512));
    uint32_t* own = g.plane(color);
    const uint32_t* oth = g.plane(1 - color);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t L = (uint32_t)g.L, R = (uint32_t)rows;
    // group blocks (in-colour index / 16) fit 32 bits while L^2 / 32 <= 2^32
    const bool hi0 = (g.L * g.L / 32) <= (int64_t(1) << 32);
    if (hi0) {
        if (color == 0)
            hipLaunchKernelGGL((lut_half_kernel<true, 0>), grid, dim3(512), 0, s, own, oth, L, R, t, tbase, k0, k1,
                               tab, bk);
        else
            hipLaunchKernelGGL((lut_half_kernel<true, 1>), grid, dim3(512), 0, s, own, oth, L, R, t, tbase, k0, k1,
                               tab, bk);
    } else {
        if (color == 0)
            hipLaunchKernelGGL((lut_half_kernel<false, 0>), grid, dim3(512), 0, s, own, oth, L, R, t, tbase, k0, k1,
                               tab, bk);
        else
            hipLaunchKernelGGL((lut_half_kernel<false, 1>), grid, dim3(512), 0, s, own, oth, L, R, t, tbase, k0, k1,
                               tab, bk);
    }
    return hipGetLastError();
}

hipError_t launch_ising_half(const Geom& g, const HalfSweepArgs& a, hipStream_t s) { return launch_half(g, a, s, 0); }
hipError_t launch_bc_half(const Geom& g, const HalfSweepArgs& a, hipStream_t s) { return launch_half(g, a, s, 1); }

namespace {

// One lane stores (vector store): *p = v, or *p += v.
__global__ void set_word_kernel(uint32_t* p, uint32_t v, int add)
{
    if (threadIdx.x == 0) *p = add ? *p + v : v;
}

}  // namespace

hipError_t launch_set_word(uint32_t* p, uint32_t v, bool add, hipStream_t s)
{
    hipLaunchKernelGGL(set_word_kernel, dim3(1), dim3(64), 0, s, p, v, add ? 1 : 0);
    return hipGetLastError();
}

}  // namespace mcl
