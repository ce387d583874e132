// Initial state and half-sweep kernels for gfx950 (rows a1, a3, a4).
//
// A half-sweep updates every cell of colour c (plane P_c) from its four
// neighbours, which all live in the other plane P_{1-c} (checkerboard
// decomposition, section 3.1):
//   vertical neighbours  : same in-plane index i, rows y - 1 and y + 1;
//   horizontal neighbours: row y, indices {i - 1, i} when (y + c) is even,
//                          {i, i + 1} when it is odd (periodic in i and y).
// Each thread owns one 16-byte column vector (32 cells) and walks down a band
// of rows, keeping the other plane's rows y - 1, y, y + 1 in registers, so
// every row of both planes is read once per band (plus one halo row above
// and below the band) and every row of P_c is written once.
#include "internal.h"

namespace mcl {
namespace {

__device__ __forceinline__ uint32_t lo32(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }

// ---------------------------------------------------------------------------
// a1: initial state.  One thread per 32-bit word (8 cells) of one plane.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void init_kernel(uint32_t* __restrict__ planes, int64_t L, int64_t W,
                                                   int model, int init_state, uint32_t k0, uint32_t k1)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = 2 * L * W;
    if (g >= total) return;
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
            const Philox4 o = philox4x32_10(lo32(blk), hi32(blk), 0u, 4u, k0, k1);
            const uint32_t sel = (uint32_t)(n & 3);
            const uint32_t w = sel == 0 ? o.v0 : sel == 1 ? o.v1 : sel == 2 ? o.v2 : o.v3;
            if (model == 0)
                s = (w < 0x80000000u) ? 1 : -1;
            else
                s = (int)(((uint64_t)w * 3u) >> 32) - 1;
        }
        word |= (uint32_t)(s + 1) << (4 * j);
    }
    planes[g] = word;
}

// Accept-draw blocks for 8 consecutive in-plane cells starting at in-colour
// site index k0 (a multiple of 8): Philox blocks k0/4 and k0/4 + 1.
struct Draws8 {
    uint32_t u[8];
};

__device__ __forceinline__ Draws8 accept_draws8(uint64_t blk, uint32_t t, uint32_t color, uint32_t k0,
                                                uint32_t k1)
{
    const Philox4 a = philox4x32_10(lo32(blk), hi32(blk), t, color, k0, k1);
    const Philox4 b = philox4x32_10(lo32(blk + 1), hi32(blk + 1), t, color, k0, k1);
    Draws8 d;
    d.u[0] = a.v0; d.u[1] = a.v1; d.u[2] = a.v2; d.u[3] = a.v3;
    d.u[4] = b.v0; d.u[5] = b.v1; d.u[6] = b.v2; d.u[7] = b.v3;
    return d;
}

// ---------------------------------------------------------------------------
// a3: Ising word update (8 cells).  Cells hold n in {0, 2}, so n ^ src is 2
// for a misaligned neighbour and 0 otherwise; the per-nibble sum halved is
// the number of misaligned neighbours m.  The flip rule of section 3.2
// (always if at most two neighbours are aligned, with e^{-4 beta} if three,
// e^{-8 beta} if four) is: flip iff m + lvl >= 2, where
// lvl = [u < T4] + [u < T8] (T8 <= T4, so u < T8 implies u < T4).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ising_word(uint32_t src, uint32_t up, uint32_t dn, uint32_t mid,
                                               uint32_t hs, const Draws8& d, uint32_t T4, uint32_t T8)
{
    uint32_t lvl = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        lvl |= ((uint32_t)(d.u[j] < T4) + (uint32_t)(d.u[j] < T8)) << (4 * j);
    const uint32_t m = ((up ^ src) + (dn ^ src) + (mid ^ src) + (hs ^ src)) >> 1;
    const uint32_t f = (m + lvl + 0x66666666u) & 0x88888888u;
    return src ^ (f >> 2);
}

// ---------------------------------------------------------------------------
// a4: Blume-Capel word update (8 cells), table lookup per cell.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bc_word(uint32_t src, uint32_t up, uint32_t dn, uint32_t mid, uint32_t hs,
                                            const Draws8& d, uint32_t pbits, const uint32_t* thr,
                                            const uint32_t* always)
{
    const uint32_t sum = up + dn + mid + hs;
    uint32_t out = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t n = (src >> (4 * j)) & 0xFu;
        const uint32_t hsum = (sum >> (4 * j)) & 0xFu;
        const uint32_t b = (pbits >> j) & 1u;
        uint32_t idx = (n * 2u + b) * 9u + hsum;
        idx = idx < 53u ? idx : 53u;
        const bool acc = always[idx] != 0u || d.u[j] < thr[idx];
        uint32_t n2 = n + 1u + b;
        n2 = n2 >= 3u ? n2 - 3u : n2;
        const uint32_t nv = (n <= 2u && acc) ? n2 : n;
        out |= nv << (4 * j);
    }
    return out;
}

__device__ __forceinline__ uint32_t pick(const uint4& v, int d)
{
    return d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w;
}

template <int MODEL>
__global__ __launch_bounds__(256) void half_sweep_kernel(uint32_t* __restrict__ own, const uint32_t* __restrict__ oth,
                                                         int64_t L, int64_t rows, uint32_t color, uint32_t t,
                                                         uint32_t k0, uint32_t k1, uint32_t T4, uint32_t T8,
                                                         BCTable tbl)
{
    __shared__ uint32_t s_thr[54];
    __shared__ uint32_t s_always[54];
    if (MODEL == 1) {
        if (threadIdx.x < 54) {
            s_thr[threadIdx.x] = tbl.thr[threadIdx.x];
            s_always[threadIdx.x] = tbl.always[threadIdx.x];
        }
        __syncthreads();
    }
    const int64_t Q = L >> 6;
    const int64_t W = L >> 4;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t q = g % Q;
    const int64_t band = g / Q;
    const int64_t y0 = band * rows;
    if (y0 >= L) return;
    const uint4* __restrict__ oth4 = reinterpret_cast<const uint4*>(oth);
    uint4* __restrict__ own4 = reinterpret_cast<uint4*>(own);
    const int64_t ym = (y0 == 0) ? L - 1 : y0 - 1;
    uint4 up = oth4[ym * Q + q];
    uint4 mid = oth4[y0 * Q + q];
    const int64_t halfL = L >> 1;
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t y = y0 + r;
        const int64_t yd = (y + 1 == L) ? 0 : y + 1;
        const uint4 dn = oth4[yd * Q + q];
        const uint4 src = own4[y * Q + q];
        const uint32_t odd = (uint32_t)((y + color) & 1);
        const int64_t hw = odd ? ((4 * q + 4 == W) ? 0 : 4 * q + 4) : ((q == 0) ? W - 1 : 4 * q - 1);
        const uint32_t halo = oth[y * W + hw];
        // in-colour index of the first cell of this vector
        const uint64_t kv = (uint64_t)(y * halfL + 32 * q);
        uint32_t pbits = 0;
        if (MODEL == 1) {
            const uint64_t pb = kv >> 7;
            const Philox4 p = philox4x32_10(lo32(pb), hi32(pb), t, 2u + color, k0, k1);
            const uint32_t sel = (uint32_t)((kv >> 5) & 3);
            pbits = sel == 0 ? p.v0 : sel == 1 ? p.v1 : sel == 2 ? p.v2 : p.v3;
        }
        uint32_t res[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t w = pick(mid, d);
            uint32_t hs;
            if (odd) {
                const uint32_t nxt = d < 3 ? pick(mid, d + 1) : halo;
                hs = funnel(nxt, w, 4);
            } else {
                const uint32_t prv = d > 0 ? pick(mid, d - 1) : halo;
                hs = funnel(w, prv, 28);
            }
            const Draws8 dr = accept_draws8((kv + 8 * d) >> 2, t, color, k0, k1);
            if (MODEL == 0)
                res[d] = ising_word(pick(src, d), pick(up, d), pick(dn, d), w, hs, dr, T4, T8);
            else
                res[d] = bc_word(pick(src, d), pick(up, d), pick(dn, d), w, hs, dr, pbits >> (8 * d), s_thr,
                                 s_always);
        }
        own4[y * Q + q] = make_uint4(res[0], res[1], res[2], res[3]);
        up = mid;
        mid = dn;
    }
}

int64_t band_rows(int64_t L)
{
    // rows per band: deep enough to amortise the two halo rows, shallow
    // enough to give the chip many thousand waves
    int64_t rows = 16;
    while (rows > 1 && (L % rows) != 0) rows >>= 1;
    return rows;
}

}  // namespace

hipError_t launch_init(const Geom& g, int model, int init_state, uint64_t seed, hipStream_t s)
{
    const int64_t total = 2 * g.L * g.W;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(init_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, g.plane0, g.L, g.W, model,
                       init_state, (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

static hipError_t launch_half(const Geom& g, const HalfSweepArgs& a, hipStream_t s, int model)
{
    const int64_t rows = band_rows(g.L);
    const int64_t threads = g.Q * (g.L / rows);
    const int64_t blocks = (threads + 255) / 256;
    BCTable tbl{};
    if (a.bc) tbl = *a.bc;
    uint32_t* own = g.plane(a.color);
    const uint32_t* oth = g.plane(1 - a.color);
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    if (model == 0)
        hipLaunchKernelGGL(half_sweep_kernel<0>, dim3((uint32_t)blocks), dim3(256), 0, s, own, oth, g.L, rows,
                           (uint32_t)a.color, a.t, k0, k1, a.T4, a.T8, tbl);
    else
        hipLaunchKernelGGL(half_sweep_kernel<1>, dim3((uint32_t)blocks), dim3(256), 0, s, own, oth, g.L, rows,
                           (uint32_t)a.color, a.t, k0, k1, a.T4, a.T8, tbl);
    return hipGetLastError();
}

hipError_t launch_ising_half(const Geom& g, const HalfSweepArgs& a, hipStream_t s) { return launch_half(g, a, s, 0); }
hipError_t launch_bc_half(const Geom& g, const HalfSweepArgs& a, hipStream_t s) { return launch_half(g, a, s, 1); }

}  // namespace mcl
