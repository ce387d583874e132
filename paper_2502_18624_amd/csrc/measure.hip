// Measurement kernels for gfx950 (rows a6, a7).
//
// Energy-like sums.  Every bond of the periodic lattice joins a colour-0 and
// a colour-1 site (L even), so the bond sum B is the sum over colour-0 cells
// of s times the sum of its four neighbours; products of two cells are
// counted eight at a time with popcounts (cell n = s + 1: a product is
// nonzero iff neither cell is 1, and +1 iff bit 1 agrees).
//
// Correlations (section 3.3).  For a source at (x, y) in plane c:
//   along y the partner (x, y + r) is in plane c ^ (r & 1), row y + r, same
//   in-plane index, so whole words pair up;
//   along x the partner (x + r, y) is in plane c ^ (r & 1) at in-plane index
//   i + m with m = r / 2 (r even) or (r - 1) / 2 + ((y + c) & 1) (r odd), a
//   funnel shift of two neighbouring words.
// The sampled sources (x = y = 0 mod 16) are cell 0 of every word of the
// rows y = 0 mod 16 of plane 0.
#include "internal.h"

namespace mcl {
namespace {

__global__ void zero_kernel(int64_t* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__device__ __forceinline__ void cell_counts(uint32_t w, int64_t& np1, int64_t& nm1, int64_t& n0, int64_t& ninv)
{
    const uint32_t b1 = w >> 1, b2 = w >> 2, b3 = w >> 3;
    const uint32_t high = (b2 | b3);
    const uint32_t m1 = ~(w | b1 | high) & 0x11111111u;
    const uint32_t z = (w & ~(b1 | high)) & 0x11111111u;
    const uint32_t p1 = (b1 & ~w & ~high) & 0x11111111u;
    const uint32_t a = popc(p1), b = popc(m1), c = popc(z);
    np1 += a;
    nm1 += b;
    n0 += c;
    ninv += 8 - (a + b + c);
}

__device__ __forceinline__ uint32_t pick(const uint4& v, int d)
{
    return d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w;
}

__global__ __launch_bounds__(256) void bmq_kernel(const uint32_t* __restrict__ p0, const uint32_t* __restrict__ p1,
                                                  int64_t L, int64_t rows, int64_t* __restrict__ acc)
{
    const int64_t Q = L >> 6, W = L >> 4;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t q = g % Q;
    const int64_t band = g / Q;
    const int64_t y0 = band * rows;
    int64_t B = 0, np1 = 0, nm1 = 0, n0 = 0, ninv = 0;
    if (y0 < L) {
        const uint4* a4 = reinterpret_cast<const uint4*>(p0);
        const uint4* b4 = reinterpret_cast<const uint4*>(p1);
        for (int64_t r = 0; r < rows; ++r) {
            const int64_t y = y0 + r;
            const int64_t yu = (y == 0) ? L - 1 : y - 1;
            const int64_t yd = (y + 1 == L) ? 0 : y + 1;
            const uint4 own = a4[y * Q + q];
            const uint4 mid = b4[y * Q + q];
            const uint4 up = b4[yu * Q + q];
            const uint4 dn = b4[yd * Q + q];
            const uint32_t odd = (uint32_t)(y & 1);
            const int64_t hw = odd ? ((4 * q + 4 == W) ? 0 : 4 * q + 4) : ((q == 0) ? W - 1 : 4 * q - 1);
            const uint32_t halo = p1[y * W + hw];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const uint32_t w = pick(mid, d);
                uint32_t hs;
                if (odd)
                    hs = funnel(d < 3 ? pick(mid, d + 1) : halo, w, 4);
                else
                    hs = funnel(w, d > 0 ? pick(mid, d - 1) : halo, 28);
                const uint32_t o = pick(own, d);
                B += pair_products(o, pick(up, d)) + pair_products(o, pick(dn, d)) + pair_products(o, w) +
                     pair_products(o, hs);
                cell_counts(o, np1, nm1, n0, ninv);
                cell_counts(w, np1, nm1, n0, ninv);
            }
        }
    }
    B = wave_sum(B);
    np1 = wave_sum(np1);
    nm1 = wave_sum(nm1);
    n0 = wave_sum(n0);
    ninv = wave_sum(ninv);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd((unsigned long long*)&acc[0], (unsigned long long)B);
        atomicAdd((unsigned long long*)&acc[1], (unsigned long long)(np1 - nm1));
        atomicAdd((unsigned long long*)&acc[2], (unsigned long long)np1);
        atomicAdd((unsigned long long*)&acc[3], (unsigned long long)nm1);
        atomicAdd((unsigned long long*)&acc[4], (unsigned long long)n0);
        atomicAdd((unsigned long long*)&acc[5], (unsigned long long)ninv);
    }
}

constexpr int kRChunk = 16;

__device__ __forceinline__ uint32_t wrap(uint32_t v, uint32_t n) { return v >= n ? v - n : v; }

// Word of cells i + m .. i + m + 7 (periodic in the row of W words), where
// cell i is cell 0 of word wd; m < 8 W.
__device__ __forceinline__ uint32_t shifted_word(const uint32_t* __restrict__ row, uint32_t W, uint32_t wd, uint32_t m)
{
    const uint32_t w0 = wrap(wd + (m >> 3), W);
    const uint32_t w1 = wrap(w0 + 1, W);
    return funnel(row[w1], row[w0], 4 * (m & 7));
}

// Every source: one thread per (plane, band of rows, 16-byte column), a
// chunk of up to kRChunk distances per grid row.
__global__ __launch_bounds__(256) void corr_all_kernel(const uint32_t* __restrict__ planes, uint32_t L, uint32_t rows,
                                                       const int32_t* __restrict__ rlist, int nr,
                                                       int64_t* __restrict__ Cx, int64_t* __restrict__ Cy)
{
    const uint32_t Q = L >> 6, W = L >> 4;
    const int j0 = blockIdx.y * kRChunk;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t q = g % Q;
    const uint32_t rest = g / Q;
    const uint32_t nbands = L / rows;
    const uint32_t c = rest / nbands;
    const uint32_t band = rest - c * nbands;
    const size_t plane_words = (size_t)L * W;
    int cx[kRChunk], cy[kRChunk];
#pragma unroll
    for (int j = 0; j < kRChunk; ++j) cx[j] = cy[j] = 0;
    if (c < 2) {
        const uint32_t* own = planes + (c ? plane_words : 0);
        for (uint32_t rr = 0; rr < rows; ++rr) {
            const uint32_t y = band * rows + rr;
            const uint4 v = reinterpret_cast<const uint4*>(own)[(size_t)y * Q + q];
            const uint32_t par = (y + c) & 1u;
#pragma unroll
            for (int j = 0; j < kRChunk; ++j) {
                if (j0 + j < nr) {
                    const uint32_t r = (uint32_t)rlist[j0 + j];
                    const uint32_t pc = c ^ (r & 1u);
                    const uint32_t* pl = planes + (pc ? plane_words : 0);
                    const uint32_t yr = wrap(y + r, L);
                    const uint4 py = reinterpret_cast<const uint4*>(pl)[(size_t)yr * Q + q];
                    const uint32_t m = (r & 1u) ? ((r - 1) >> 1) + par : (r >> 1);
                    const uint32_t* prow = pl + (size_t)y * W;
                    int sx = 0, sy = 0;
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const uint32_t o = pick(v, d);
                        sy += pair_products(o, pick(py, d));
                        sx += pair_products(o, shifted_word(prow, W, 4 * q + d, m));
                    }
                    cx[j] += sx;
                    cy[j] += sy;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kRChunk; ++j) {
        const int sx = wave_sum_i32(cx[j]);
        const int sy = wave_sum_i32(cy[j]);
        if ((threadIdx.x & 63) == 0 && j0 + j < nr) {
            atomicAdd((unsigned long long*)&Cx[j0 + j], (unsigned long long)(int64_t)sx);
            atomicAdd((unsigned long long*)&Cy[j0 + j], (unsigned long long)(int64_t)sy);
        }
    }
}

// Sampled sources (x = y = 0 mod 16): cell 0 of word a of plane 0, row 16 b.
// Partners: along x (16 a + r, 16 b) is cell (8 a + r / 2) mod (L / 2) of
// row 16 b in plane r & 1; along y (16 a, 16 b + r) is cell 0 of word a of
// row 16 b + r in plane r & 1.  Block order puts the distance chunks of one
// band of source rows next to each other so their partner rows are shared
// in cache.
__global__ __launch_bounds__(256) void corr_sampled_kernel(const uint32_t* __restrict__ planes, uint32_t L,
                                                           uint32_t brows, uint32_t ablocks, uint32_t nchunks,
                                                           const int32_t* __restrict__ rlist, int nr,
                                                           int64_t* __restrict__ Cx, int64_t* __restrict__ Cy)
{
    const uint32_t W = L >> 4;       // words per row = number of source columns
    const uint32_t nb = L >> 4;      // number of source rows
    const uint32_t half = L >> 1;
    const size_t plane_words = (size_t)L * W;
    const uint32_t ab = blockIdx.x % ablocks;
    const uint32_t chunk = (blockIdx.x / ablocks) % nchunks;
    const uint32_t band = blockIdx.x / (ablocks * nchunks);
    const int j0 = (int)chunk * kRChunk;
    const uint32_t a = ab * blockDim.x + threadIdx.x;
    int cx[kRChunk], cy[kRChunk];
#pragma unroll
    for (int j = 0; j < kRChunk; ++j) cx[j] = cy[j] = 0;
    if (a < W && band * brows < nb) {
        for (uint32_t bb = 0; bb < brows; ++bb) {
            const uint32_t y = 16u * (band * brows + bb);
            const int src = (int)(planes[(size_t)y * W + a] & 0xFu) - 1;
#pragma unroll
            for (int j = 0; j < kRChunk; ++j) {
                if (j0 + j < nr) {
                    const uint32_t r = (uint32_t)rlist[j0 + j];
                    const uint32_t* pl = planes + ((r & 1u) ? plane_words : 0);
                    const uint32_t i = wrap(8u * a + (r >> 1), half);
                    const int px = (int)((pl[(size_t)y * W + (i >> 3)] >> (4 * (i & 7))) & 0xFu) - 1;
                    const uint32_t yr = wrap(y + r, L);
                    const int py = (int)(pl[(size_t)yr * W + a] & 0xFu) - 1;
                    cx[j] += src * px;
                    cy[j] += src * py;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kRChunk; ++j) {
        const int sx = wave_sum_i32(cx[j]);
        const int sy = wave_sum_i32(cy[j]);
        if ((threadIdx.x & 63) == 0 && j0 + j < nr) {
            atomicAdd((unsigned long long*)&Cx[j0 + j], (unsigned long long)(int64_t)sx);
            atomicAdd((unsigned long long*)&Cy[j0 + j], (unsigned long long)(int64_t)sy);
        }
    }
}

int64_t pick_rows(int64_t L, int64_t want)
{
    int64_t rows = want;
    while (rows > 1 && (L % rows) != 0) rows >>= 1;
    return rows;
}

}  // namespace

hipError_t launch_zero(int64_t* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_bmq(const Geom& g, int64_t* acc, hipStream_t s)
{
    const int64_t rows = pick_rows(g.L, 16);
    const int64_t threads = g.Q * (g.L / rows);
    hipLaunchKernelGGL(bmq_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, g.plane(0), g.plane(1),
                       g.L, rows, acc);
    return hipGetLastError();
}

hipError_t launch_corr_all(const Geom& g, const int32_t* r_dev, int nr, int64_t* Cx, int64_t* Cy, hipStream_t s)
{
    if (nr <= 0) return hipSuccess;
    const int64_t rows = pick_rows(g.L, 16);
    const int64_t threads = 2 * g.Q * (g.L / rows);
    const uint32_t chunks = (uint32_t)((nr + kRChunk - 1) / kRChunk);
    hipLaunchKernelGGL(corr_all_kernel, dim3((uint32_t)((threads + 255) / 256), chunks), dim3(256), 0, s, g.plane0,
                       (uint32_t)g.L, (uint32_t)rows, r_dev, nr, Cx, Cy);
    return hipGetLastError();
}

hipError_t launch_corr_sampled(const Geom& g, const int32_t* r_dev, int nr, int64_t* Cx, int64_t* Cy, hipStream_t s)
{
    if (nr <= 0) return hipSuccess;
    const int64_t nb = g.L / 16;
    const int64_t brows = pick_rows(nb, 8);
    const uint32_t ablocks = (uint32_t)((g.W + 255) / 256);
    const uint32_t chunks = (uint32_t)((nr + kRChunk - 1) / kRChunk);
    const int64_t blocks = (int64_t)ablocks * chunks * (nb / brows);
    hipLaunchKernelGGL(corr_sampled_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, g.plane0, (uint32_t)g.L,
                       (uint32_t)brows, ablocks, chunks, r_dev, nr, Cx, Cy);
    return hipGetLastError();
}

}  // namespace mcl
