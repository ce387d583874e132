// Measurement kernels for gfx950: B, M, Q, counts and the Schwinger-Dyson
// histogram; the correlation sums of section 3.3.
//
// Energy-like sums.  Every bond of the periodic lattice joins a colour-0 and
// a colour-1 site (L even), so the bond sum B is the sum over colour-0 cells
// of s times the sum of its four neighbours; products of two cells are
// counted eight at a time with popcounts (cell n = s + 1: a product is
// nonzero iff neither cell is 1, and +1 iff bit 1 agrees; Ising cells are
// never 1, so there a word pair needs one xor-and and one popcount).
//
// Correlations (section 3.3).  For a source at (x, y) in plane c:
//   along y the partner (x, y + r) is in plane c ^ (r & 1), row y + r, same
//   in-plane index, so whole words pair up;
//   along x the partner (x + r, y) is in plane c ^ (r & 1) at in-plane index
//   i + m with m = r / 2 (r even) or (r - 1) / 2 + ((y + c) & 1) (r odd), a
//   funnel shift of two neighbouring words.
// Every-source distances r <= 32 run from an LDS tile of both planes with 32
// halo rows; longer every-source distances (full mode) read partners from
// global memory.  The sampled sources (x = y = 0 mod 16) are cell 0 of
// every word of the rows y = 0 mod 16 of plane 0: along x each source row is
// unpacked to one int8 per site in LDS; along y the work runs over target
// rows against a compact int8 copy of the sources, four products per dot4.
#include <algorithm>
#include <cstdlib>

#include "internal.h"

namespace mcl {
namespace {

__global__ void zero_kernel(int64_t* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__device__ __forceinline__ uint32_t pick(const uint4& v, int d)
{
    return d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w;
}

__device__ __forceinline__ uint32_t wrap(uint32_t v, uint32_t n) { return v >= n ? v - n : v; }

// acc + (number of set bits of x) as one v_bcnt_u32_b32.  Written out, sums
// of several bit counts are re-associated into separate counts and
// three-input adds.
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc)
{
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// Per-word cell counts: +1 (n = 2), -1 (n = 0), 0 (n = 1); anything else is
// what they leave.  Bit 0 of each nibble carries the test; the mask of the
// other bits is folded into `high`, so each count is one three-input
// logic operation and one bit count.
__device__ __forceinline__ void cell_counts(uint32_t w, uint32_t& np1, uint32_t& nm1, uint32_t& n0)
{
    const uint32_t b1 = w >> 1, high = (w >> 2) | (w >> 3) | 0xEEEEEEEEu;
    np1 = bcnt_acc(b1 & ~w & ~high, np1);
    nm1 = bcnt_acc(~(w | b1 | high), nm1);
    n0 = bcnt_acc(w & ~(b1 | high), n0);
}

// Sum of s * s' over the 8 cell pairs of two words, as (nonzero pairs,
// pairs of opposite sign): the sum is nz - 2 * diff.
__device__ __forceinline__ void pair_counts(uint32_t a, uint32_t b, uint32_t& nz, uint32_t& diff)
{
    const uint32_t z = ~(a | b) & 0x11111111u;
    nz = bcnt_acc(z, nz);
    diff = bcnt_acc(((a ^ b) >> 1) & z, diff);
}

// Cell width traits: 4-bit cells (n = s + 1, 8 per word) and 1-bit cells
// (bit = [s > 0], Ising only, 32 per word).
template <int CB>
struct Cell;

template <>
struct Cell<4> {
    static constexpr int kPerWord = 8;
    static constexpr int kVecShift = 6;     // 16-byte vectors per row = L >> 6
    static constexpr int kWordShift = 4;    // words per row = L >> 4
    static __device__ __forceinline__ void pair(uint32_t a, uint32_t b, uint32_t& nz, uint32_t& diff)
    {
        pair_counts(a, b, nz, diff);
    }
    static __device__ __forceinline__ void counts(uint32_t w, uint32_t& np1, uint32_t& nm1, uint32_t& n0)
    {
        cell_counts(w, np1, nm1, n0);
    }
    // neighbour word of cells i - 1 (even) / i + 1 (odd)
    static __device__ __forceinline__ uint32_t left(uint32_t w, uint32_t prev) { return funnel(w, prev, 28); }
    static __device__ __forceinline__ uint32_t right(uint32_t next, uint32_t w) { return funnel(next, w, 4); }
    static __device__ __forceinline__ int spin(const uint32_t* __restrict__ row, uint32_t i)
    {
        return (int)((row[i >> 3] >> (4 * (i & 7))) & 0xFu) - 1;
    }
};

template <>
struct Cell<1> {
    static constexpr int kPerWord = 32;
    static constexpr int kVecShift = 8;
    static constexpr int kWordShift = 6;
    static __device__ __forceinline__ void pair(uint32_t a, uint32_t b, uint32_t& nz, uint32_t& diff)
    {
        nz += 32;
        diff = bcnt_acc(a ^ b, diff);
    }
    // -1 cells: what the +1 cells leave (taken at the end of the pass)
    static __device__ __forceinline__ void counts(uint32_t w, uint32_t& np1, uint32_t&, uint32_t&)
    {
        np1 = bcnt_acc(w, np1);
    }
    static __device__ __forceinline__ uint32_t left(uint32_t w, uint32_t prev) { return funnel(w, prev, 31); }
    static __device__ __forceinline__ uint32_t right(uint32_t next, uint32_t w) { return funnel(next, w, 1); }
    static __device__ __forceinline__ int spin(const uint32_t* __restrict__ row, uint32_t i)
    {
        return ((row[i >> 5] >> (i & 31)) & 1u) ? 1 : -1;
    }
};

// Sum v[0..N) over the workgroup (wave sums, then across the waves in LDS)
// and add the totals to out[0..N): one atomic per value per workgroup, so
// the device-wide atomics on a handful of addresses stay few.
template <int N>
__device__ __forceinline__ void block_add(const int64_t (&v)[N], int64_t* __restrict__ out, int64_t (*lds)[N])
{
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int64_t s = wave_sum(v[i]);
        if ((threadIdx.x & 63) == 0) lds[wave][i] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        int64_t tot = 0;
        for (int w = 0; w < nwaves; ++w) tot += lds[w][i];
        if (tot != 0) atomicAdd((unsigned long long*)&out[i], (unsigned long long)tot);
    }
    __syncthreads();
}

// As block_add for 2 N values: v[0..N) go to X, v[N..2N) to Y.
template <int N>
__device__ __forceinline__ void block_add_xy(const int64_t (&v)[2 * N], int64_t* __restrict__ X,
                                             int64_t* __restrict__ Y, int64_t (*lds)[2 * N])
{
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < 2 * N; ++i) {
        const int64_t s = wave_sum(v[i]);
        if ((threadIdx.x & 63) == 0) lds[wave][i] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
        int64_t tot = 0;
        for (int w = 0; w < nwaves; ++w) tot += lds[w][i];
        int64_t* dst = i < N ? &X[i] : &Y[i - N];
        if (tot != 0) atomicAdd((unsigned long long*)dst, (unsigned long long)tot);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// B, M, Q, counts.  One thread per 16-byte column of plane 0, walking a
// band of rows with plane 1's rows y - 1, y, y + 1 in registers.
// ---------------------------------------------------------------------------
// Histogram of t = sigma h + 4 (0..8) over the cells of word o, whose four
// neighbour words are a, b (vertical), c (same row) and d (horizontal).
// 4-bit cells: the neighbour sum S = sum n = h + 4 fits a nibble, and
// t = 4 for sigma = 0, S for sigma = +1, 8 - S for sigma = -1.
__device__ __forceinline__ void sd_add4(uint32_t o, uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t (&hist)[9])
{
    const uint32_t S = a + b + c + d;
    const uint32_t e2 = (o >> 1) & 0x11111111u, e0 = ~(o | (o >> 1)) & 0x11111111u;
    const uint32_t m2 = shl_opaque<4>(e2) - e2;                    // 0xF where sigma = +1
    const uint32_t m0 = shl_opaque<4>(e0) - e0;                    // 0xF where sigma = -1
    const uint32_t t = (S & m2) | ((0x88888888u - S) & m0) | (0x44444444u & ~(m0 | m2));
    const uint32_t b0 = t & 0x11111111u, b1 = (t >> 1) & 0x11111111u;
    const uint32_t b2 = (t >> 2) & 0x11111111u, b3 = (t >> 3) & 0x11111111u;
    const uint32_t n0 = b0 ^ 0x11111111u, n1 = b1 ^ 0x11111111u, n2 = b2 ^ 0x11111111u, n3 = b3 ^ 0x11111111u;
    const uint32_t lo[4] = {n0 & n1, b0 & n1, n0 & b1, b0 & b1};
    const uint32_t hi0 = n2 & n3, hi1 = b2 & n3;
#pragma unroll
    for (int v = 0; v < 8; ++v) hist[v] = bcnt_acc(lo[v & 3] & (v < 4 ? hi0 : hi1), hist[v]);
    hist[8] = bcnt_acc(b3, hist[8]);
}

// 1-bit cells: t = 2 (aligned neighbours), from the four words of
// differences d_j = neighbour ^ own.
__device__ __forceinline__ void sd_add1(uint32_t o, uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t (&hist)[9])
{
    const uint32_t d0 = a ^ o, d1 = b ^ o, d2 = c ^ o, d3 = d ^ o;
    const uint32_t t1 = d0 ^ d1, t2 = d2 ^ d3;
    const uint32_t all_eq = ~(d0 | d1 | d2 | d3);                    // 4 aligned: t = 8
    const uint32_t all_ne = d0 & d1 & d2 & d3;                       // 0 aligned: t = 0
    const uint32_t one_ne = (t1 ^ t2) & ~((d0 & d1) | (d2 & d3));    // 3 aligned: t = 6
    const uint32_t one_eq = (t1 ^ t2) & (d0 | d1) & (d2 | d3);       // 1 aligned: t = 2
    hist[8] = bcnt_acc(all_eq, hist[8]);
    hist[0] = bcnt_acc(all_ne, hist[0]);
    hist[6] = bcnt_acc(one_ne, hist[6]);
    hist[2] = bcnt_acc(one_eq, hist[2]);
    // two aligned (t = 4): the rest of the cells, at the end of the pass
}

// 4-bit Ising cells (n in {0, 2}): per nibble S = 2 d, d the number of
// neighbours of the opposite sign, 0..4 (each xor nibble is 0 or 2, their
// sum at most 8), so bits 1, 2, 3 of the nibble are bits 0, 1, 2 of d.
// With n_k the number of cells with d = k, adds to
//   e[0] the set bits of S:            n_1 + n_2 + 2 n_3 + n_4,
//   e[1] those at nibble bit 1:        n_1 + n_3,
//   e[2] bits 1 and 2 both set:        n_3,
//   e[3] those at nibble bit 3:        n_4,
// from which the end of the pass takes n_1 .. n_4; n_0 is the rest of the
// cells, and the bond sum follows from the histogram.
__device__ __forceinline__ void sd_add_ising4(uint32_t o, uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                              uint32_t (&e)[4])
{
    const uint32_t S = xad(d, o, xad(c, o, xad(b, o, a ^ o)));
    e[0] = bcnt_acc(S, e[0]);
    e[1] = bcnt_acc(S & 0x22222222u, e[1]);
    e[2] = bcnt_acc(S & (S << 1) & 0x44444444u, e[2]);
    e[3] = bcnt_acc(S & 0x88888888u, e[3]);
}

// T bits (the sampled columns, see below) of row y from the thread's
// vector v of the row's colour-(y & 1) plane: 4-bit cells, vector q holds
// the cells 8 a for a = 4 q .. 4 q + 3 at nibble 0 of its words, and 8 lanes
// make one word; 1-bit cells, vector q holds a = 16 q .. 16 q + 15 at bits
// 0, 8, 16, 24 of its words, and 2 lanes make one word.  The lanes of a
// word share the row (Q is a multiple of 8, resp. 2, from L = 512 on).
template <int MODEL>
__device__ __forceinline__ void emit_tbits(const uint4& v, uint32_t q, uint32_t y, uint32_t L,
                                           uint32_t* __restrict__ tb)
{
    const uint32_t NSW = L >> 9;
    if (MODEL == 2) {
        uint32_t bits = 0;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t x = pick(v, d) & 0x01010101u;
            bits |= ((x | (x >> 7) | (x >> 14) | (x >> 21)) & 0xFu) << (4 * d);
        }
        uint32_t w = bits << (16u * (q & 1u));
        w |= __shfl_xor(w, 1);
        if ((q & 1u) == 0) tb[(size_t)y * NSW + (q >> 1)] = w;
        return;
    }
    uint32_t sb = 0, zb = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        sb |= ((pick(v, d) >> 1) & 1u) << d;       // n = 2: s = +1
        zb |= ((~pick(v, d)) & 1u) << d;           // n != 1: s != 0
    }
    const uint32_t sh = 4u * (q & 7u);
    uint32_t ws = sb << sh, wz = zb << sh;
    ws |= __shfl_xor(ws, 1);
    ws |= __shfl_xor(ws, 2);
    ws |= __shfl_xor(ws, 4);
    if (MODEL == 1) {
        wz |= __shfl_xor(wz, 1);
        wz |= __shfl_xor(wz, 2);
        wz |= __shfl_xor(wz, 4);
    }
    if ((q & 7u) == 0) {
        tb[(size_t)y * NSW + (q >> 3)] = ws;
        if (MODEL == 1) tb[(size_t)(L + y) * NSW + (q >> 3)] = wz;
    }
}

// v of lane i + 1 (from_right) or lane i - 1 (from_left) of the wave, by a
// DPP wave shift; the lane at the end without a neighbour gets an
// unspecified value.
__device__ __forceinline__ uint32_t from_right(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, false);    // wave_shl:1
}
__device__ __forceinline__ uint32_t from_left(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, false);    // wave_shr:1
}

// One pass over both planes: B and M, Q and the value counts, and the
// Schwinger-Dyson histogram (section 4) of sigma h over every site; with tb
// set (L >= 512), also the T bits of every row.  A task is a column vector
// q of a band of rows; the thread keeps rows y - 1, y, y + 1 of both
// planes.  Colour-0 sites carry the bonds (each bond has one colour-0
// end); both colours add to the counts and the histogram.
// WAVE_ROWS: L / (cells per vector) is a multiple of 64, so the 64 lanes of
// a wave share their band and its row parity is a scalar.
template <int MODEL, bool WAVE_ROWS>
__global__ __launch_bounds__(256) void bmq_kernel(const uint32_t* __restrict__ p0, const uint32_t* __restrict__ p1,
                                                  uint32_t L, uint32_t rows, int64_t* __restrict__ acc,
                                                  uint32_t* __restrict__ tb)
{
    constexpr int CB = MODEL == 2 ? 1 : 4;
    using C = Cell<CB>;
    __shared__ int64_t red[4][14];
    const uint32_t Q = L >> C::kVecShift, W = L >> C::kWordShift;
    const uint32_t tasks = Q * (L / rows);
    uint32_t nz = 0, diff = 0, np1 = 0, nm1 = 0, n0 = 0, cells = 0;
    uint32_t hist[9], e[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 9; ++k) hist[k] = 0;
    // workgroup ids go round-robin to the 8 XCDs: XCD x takes the x-th
    // eighth of the workgroups in order, so the tasks beside a workgroup's
    // (the rest of its bands, the bands above and below) run on the same
    // XCD at about the same time and the lines they share meet in its L2
    const uint32_t nb = gridDim.x;
    const uint32_t blk = (nb & 7u) == 0 ? (blockIdx.x & 7u) * (nb >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    for (uint32_t g = blk * blockDim.x + threadIdx.x; g < tasks; g += nb * blockDim.x) {
        const uint32_t q = g % Q;
        uint32_t y0 = (g / Q) * rows;
        if (WAVE_ROWS) y0 = __builtin_amdgcn_readfirstlane(y0);
        const uint4* a4 = reinterpret_cast<const uint4*>(p0) + q;
        const uint4* b4 = reinterpret_cast<const uint4*>(p1) + q;
        const size_t yu = y0 == 0 ? L - 1 : y0 - 1;
        uint4 aup = a4[yu * Q], amid = a4[(size_t)y0 * Q];
        uint4 bup = b4[yu * Q], bmid = b4[(size_t)y0 * Q];
        const uint32_t hwl = (q == 0) ? W - 1 : 4 * q - 1;
        const uint32_t hwr = (4 * q + 4 == W) ? 0 : 4 * q + 4;
        // the words beside the vector are the neighbouring lanes' end words
        // (moved across by DPP), except at the ends of the wave or the row
        const uint32_t lane = threadIdx.x & 63u;
        const bool edge_l = lane == 0 || q == 0, edge_r = lane == 63 || q + 1 == Q;
        cells += 2 * C::kPerWord * 4 * rows;    // both planes, 4 words a row
        for (uint32_t r = 0; r < rows; ++r) {
            const uint32_t y = y0 + r;
            const size_t yd = (y + 1 == L) ? 0 : y + 1;
            const uint4 adn = a4[yd * Q], bdn = b4[yd * Q];
            const bool odd = (y & 1u) != 0;      // colour-0 sites of row y have x = 2 i + (y & 1)
            if (tb) emit_tbits<MODEL>(odd ? bmid : amid, q, y, L, tb);
            // colour 0 looks right (i + 1) on odd rows, colour 1 on even rows
            uint32_t bhalo = odd ? from_right(bmid.x) : from_left(bmid.w);
            uint32_t ahalo = odd ? from_left(amid.w) : from_right(amid.x);
            if (odd ? edge_r : edge_l) bhalo = p1[(size_t)y * W + (odd ? hwr : hwl)];
            if (odd ? edge_l : edge_r) ahalo = p0[(size_t)y * W + (odd ? hwl : hwr)];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const uint32_t wb = pick(bmid, d), wa = pick(amid, d);
                const uint32_t hb = odd ? C::right(d < 3 ? pick(bmid, d + 1) : bhalo, wb)
                                        : C::left(wb, d > 0 ? pick(bmid, d - 1) : bhalo);
                const uint32_t ha = odd ? C::left(wa, d > 0 ? pick(amid, d - 1) : ahalo)
                                        : C::right(d < 3 ? pick(amid, d + 1) : ahalo, wa);
                C::counts(wa, np1, nm1, n0);
                C::counts(wb, np1, nm1, n0);
                if (MODEL == 0) {
                    sd_add_ising4(wa, pick(bup, d), pick(bdn, d), wb, hb, e);
                    sd_add_ising4(wb, pick(aup, d), pick(adn, d), wa, ha, e);
                    continue;
                }
                C::pair(wa, pick(bup, d), nz, diff);
                C::pair(wa, pick(bdn, d), nz, diff);
                C::pair(wa, wb, nz, diff);
                C::pair(wa, hb, nz, diff);
                if (CB == 4) {
                    sd_add4(wa, pick(bup, d), pick(bdn, d), wb, hb, hist);
                    sd_add4(wb, pick(aup, d), pick(adn, d), wa, ha, hist);
                } else {
                    sd_add1(wa, pick(bup, d), pick(bdn, d), wb, hb, hist);
                    sd_add1(wb, pick(aup, d), pick(adn, d), wa, ha, hist);
                }
            }
            aup = amid;
            amid = adn;
            bup = bmid;
            bmid = bdn;
        }
    }
    if (MODEL == 0) {
        // n_1 .. n_4 from the sums of sd_add_ising4 (t = 8 - 2 d); the
        // thread's cells were 16 per word pair, the rest of the histogram
        // has d = 0; each bond is seen from both ends, so the bond sum is
        // 2 (cells) - sum of d over all cells
        hist[2] = e[2];
        hist[0] = e[3];
        hist[6] = e[1] - e[2];
        hist[4] = e[0] - e[1] - e[2] - e[3];
        hist[8] = cells - hist[6] - hist[4] - hist[2] - hist[0];
        nz = 2 * cells;
        diff = 0;
        const uint32_t dsum = hist[6] + 2 * hist[4] + 3 * hist[2] + 4 * hist[0];
        nz -= dsum;
    }
    if (MODEL == 2) {
        // 1-bit cells are all +1 or -1; t = 4 is what the other bins leave
        nm1 = cells - np1;
        hist[4] = cells - hist[0] - hist[2] - hist[6] - hist[8];
    }
    // acc: [0] B, [1] M, [2] #(+1), [3] #(-1), [4] #(0), [5 + k] #(sigma h = k - 4);
    // invalid cells are what the three counts leave of L^2 (done on the host)
    int64_t v[14] = {(int64_t)nz - 2 * (int64_t)diff, (int64_t)np1 - (int64_t)nm1, (int64_t)np1, (int64_t)nm1,
                     (int64_t)n0};
#pragma unroll
    for (int k = 0; k < 9; ++k) v[5 + k] = (int64_t)hist[k];
    block_add<14>(v, acc, red);
}

// ---------------------------------------------------------------------------
// Correlations, every source, r = 0..R (R <= 32): LDS tile of SW words (+1 halo word
// on the right for x-partners, +1 on the left for the B/M/Q work) by TH
// source rows (+32 halo rows below for y-partners), both planes, with the
// cells as 1-bit words of 32 cells: the sign bit for Ising, and for
// Blume-Capel a second word of nonzero bits.  A 4-bit row vector (32 cells)
// packs into one word, a 1-bit plane word is stored as it is, so every
// model has L / 64 words per tile row.  Thread (j, g) handles word column j
// and rows 16 g .. 16 g + 15 of the tile along one axis, for r in
// [RLO, RHI]: per distance, axis and 32 pairs one funnel shift (x only),
// an xor (and two ands for Blume-Capel) and the bit counts.  For 4-bit
// Ising lattices the same tiles also give the B/M/Q sums (tile_bmq), which
// would otherwise read the 4-bit lattice a second time.
// ---------------------------------------------------------------------------
constexpr int kSW = 32;
constexpr int kTH = 64;
constexpr int kHalo = 32;
constexpr int kTileRows = kTH + kHalo;

// Tile columns: the strip's words 0 .. kSW - 1 at CO .. CO + kSW - 1, the
// word right of the strip after them, and with LEFT (CO = 1) the word left
// of it at column 0 (of which only the last cell is loaded).
template <int MODEL, bool LEFT>
struct ShortTile {
    static constexpr int NB = MODEL == 1 ? 2 : 1;   // bit planes: sign [, nonzero]
    static constexpr int CO = LEFT ? 1 : 0;
    static constexpr int COLS = kSW + 1 + CO;
    uint32_t v[2][NB][kTileRows][COLS];
};

// Bit `BIT` (0 or 1) of each nibble of the 4 words (32 cells), in cell
// order: bit 8 d + k of the result is nibble k of word d.  The words are
// first interleaved (bit 4 k + d = nibble k of word d: one shift and one bit
// select each), then the bit index is rotated from (k, d) to (d, k) by three
// swaps of index bits (0 with 2, 1 with 3, 2 with 4) and a byte permutation
// (3 with 4).
template <int S, uint32_t M>
__device__ __forceinline__ uint32_t delta_swap(uint32_t x)
{
    const uint32_t t = ((x >> S) ^ x) & M;
    return x ^ t ^ (t << S);
}

__device__ __forceinline__ uint32_t bit_select(uint32_t m, uint32_t a, uint32_t b) { return (a & m) | (b & ~m); }

template <int BIT>
__device__ __forceinline__ uint32_t nibble_bits(const uint4& v, bool invert)
{
    const uint32_t s0 = BIT ? v.x >> 1 : v.x;
    const uint32_t s1 = BIT ? v.y : v.y << 1;
    const uint32_t s2 = v.z << (2 - BIT);
    const uint32_t s3 = v.w << (3 - BIT);
    uint32_t z = bit_select(0x11111111u, s0, bit_select(0x22222222u, s1, bit_select(0x88888888u, s3, s2)));
    if (invert) z = ~z;
    z = delta_swap<3, 0x0A0A0A0Au>(z);
    z = delta_swap<6, 0x00CC00CCu>(z);
    z = delta_swap<12, 0x0000F0F0u>(z);
    return __builtin_amdgcn_perm(z, z, 0x03010200u);
}

// Column index q of a tile word, periodic in the row of Wp words (q < Wp + kSW + 1).
__device__ __forceinline__ uint32_t wrap_col(uint32_t q, uint32_t Wp)
{
    return q < Wp ? q : (Wp > (uint32_t)kSW ? q - Wp : q % Wp);
}

// Tile rows row, row + step, ... (< kTileRows) of column col (lattice word
// column qq) of both planes, as 1-bit words; tile row r is lattice row
// y0 + r, periodic (y0 + r < L + kHalo <= 2 L).  `bad` collects the bits of
// 4-bit Ising cells that hold no spin (n other than 0 and 2).
template <int MODEL, class TT>
__device__ __forceinline__ void tile_load(TT& T, const uint32_t* __restrict__ planes,
                                          const uint4* __restrict__ P4, size_t plane_units, uint32_t Wp, uint32_t L,
                                          uint32_t y0, uint32_t row, uint32_t step, uint32_t col, uint32_t qq,
                                          uint32_t& bad)
{
    constexpr int NB = TT::NB;
    uint32_t y = y0 + row;
    if (y >= L) y -= L;
    for (; row < (uint32_t)kTileRows; row += step) {
#pragma unroll
        for (uint32_t c = 0; c < 2; ++c) {
            const size_t at = c * plane_units + (size_t)y * Wp + qq;
            if (MODEL == 2) {
                T.v[c][0][row][col] = planes[at];
            } else {
                const uint4 v = P4[at];
                T.v[c][0][row][col] = nibble_bits<1>(v, false);                    // n = 2: s = +1
                if (MODEL == 1) T.v[c][NB - 1][row][col] = nibble_bits<0>(v, true);   // n != 1
                if (MODEL == 0) bad |= (v.x | v.y | v.z | v.w) & 0xDDDDDDDDu;
            }
        }
        y += step;
        if (y >= L) y -= L;
    }
}

// Column 0 of tile row `row` (lattice word column qq) of both planes, for
// 4-bit cells: the B/M/Q work uses only its last cell (the i - 1 neighbour
// of the strip's cell 0), so one 4-byte load of the vector's last word gives
// it (cell 31 is nibble 7 of that word, its sign bit bit 29).
template <class TT>
__device__ __forceinline__ void tile_load_left(TT& T, const uint4* __restrict__ P4, size_t plane_units, uint32_t Wp,
                                               uint32_t L, uint32_t y0, uint32_t row, uint32_t qq)
{
    uint32_t y = y0 + row;
    if (y >= L) y -= L;
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c) {
        const uint32_t w = reinterpret_cast<const uint32_t*>(P4 + c * plane_units + (size_t)y * Wp + qq)[3];
        T.v[c][0][row][0] = ((w >> 29) & 1u) << 31;
    }
}

// Distances [RLO, RHI] along one axis (AXIS 0: x, 1: y) for the cells of
// plane C in tile row lr (PAR: parity of y + C).
template <int MODEL, int AXIS, int RLO, int RHI, int C, int PAR, class TT>
__device__ __forceinline__ void short_row(const TT& T, int lr, int j, int (&acc)[33])
{
    constexpr int Z = TT::NB - 1;                       // plane of nonzero bits (Blume-Capel)
    const int jc = j + TT::CO;                          // the strip's word j in the tile
    const uint32_t o = T.v[C][0][lr][jc];
    const uint32_t oz = MODEL == 1 ? T.v[C][Z][lr][jc] : 0u;
    uint32_t w0[2], w1[2], z0[2], z1[2];
    if (AXIS == 0) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            w0[p] = T.v[p][0][lr][jc];
            w1[p] = T.v[p][0][lr][jc + 1];
            z0[p] = MODEL == 1 ? T.v[p][Z][lr][jc] : 0u;
            z1[p] = MODEL == 1 ? T.v[p][Z][lr][jc + 1] : 0u;
        }
    }
#pragma unroll
    for (int r = RLO; r <= RHI; ++r) {
        const int pc = C ^ (r & 1);
        uint32_t pv, pz = 0;
        if (AXIS == 0) {
            const int m = (r & 1) ? ((r - 1) >> 1) + PAR : (r >> 1);     // in-plane shift, 0..16
            pv = m ? funnel(w1[pc], w0[pc], m) : w0[pc];
            if (MODEL == 1) pz = m ? funnel(z1[pc], z0[pc], m) : z0[pc];
        } else {
            pv = T.v[pc][0][lr + r][jc];
            if (MODEL == 1) pz = T.v[pc][Z][lr + r][jc];
        }
        if (MODEL != 1) {
            acc[r] += (int)popc(o ^ pv);                // pairs of opposite sign
        } else {
            const uint32_t nz = pz & oz;
            acc[r] += (int)popc(nz) - 2 * (int)popc(nz & (o ^ pv));
        }
    }
}

// Distances [RLO, RHI] along one axis over the thread's kTH / 4 rows of the tile.
template <int MODEL, int AXIS, int RLO, int RHI, class TT>
__device__ __forceinline__ void short_chunk(const TT& T, int j, int g, int (&acc)[33])
{
    // tile rows G g .. G g + G - 1 (G = kTH / 4); the tile's first row is
    // even, so the parity of y + c is that of the local row + c
    constexpr int G = kTH / 4;
    for (int k = 0; k < G; k += 2) {
        const int lr = G * g + k;
        short_row<MODEL, AXIS, RLO, RHI, 0, 0>(T, lr, j, acc);
        short_row<MODEL, AXIS, RLO, RHI, 1, 1>(T, lr, j, acc);
        short_row<MODEL, AXIS, RLO, RHI, 0, 1>(T, lr + 1, j, acc);
        short_row<MODEL, AXIS, RLO, RHI, 1, 0>(T, lr + 1, j, acc);
    }
}

template <int MODEL, int AXIS, class TT>
__device__ __forceinline__ void short_tile(const TT& T, int j, int g, int R, int (&acc)[33])
{
    // r = 0 counts no pair of opposite sign for Ising cells (acc[0] stays 0)
    short_chunk<MODEL, AXIS, MODEL == 1 ? 0 : 1, 10>(T, j, g, acc);
    if (R > 10) short_chunk<MODEL, AXIS, 11, 21>(T, j, g, acc);
    if (R > 21) short_chunk<MODEL, AXIS, 22, 32>(T, j, g, acc);
}

// The B/M/Q pass on a tile's 1-bit words (4-bit Ising cells): the sites
// of tile rows 1 .. kTH (lattice rows y0 + 1 .. y0 + kTH, so every row once
// over the strip's tiles), word column j, both planes; the thread takes rows
// 1 + f, 9 + f, ... (f = tid / 32, so the two halves of a wave read
// adjacent rows).  Per word of 32 cells the four neighbour words (other
// plane: rows r - 1, r + 1, the same index, and index i + 1 or i - 1 by the
// parity of y + c) give the sigma-h bins as in the B/M/Q pass; the +1 cells
// are the set sign bits; the T bits of row y are bits 0, 8, 16, 24 of the
// words of plane y & 1 (the sampled columns x = 0 mod 16), merged over 8
// lanes into one word.
template <int MODEL, class TT>
__device__ __forceinline__ void tile_bmq(const TT& T, uint32_t y0, uint32_t q0, uint32_t L,
                                         uint32_t Wp, int j, uint32_t* __restrict__ tb, uint32_t (&hist)[9],
                                         uint32_t& np1, uint32_t& sites)
{
    static_assert(TT::CO == 1, "the B/M/Q work needs the word left of the strip");
    const uint32_t NSW = L >> 9;
    const int jc = j + 1;
    const bool in_strip = q0 + (uint32_t)j < Wp;
    for (uint32_t r = 1 + (threadIdx.x >> 5); r <= (uint32_t)kTH; r += 8) {
        if (in_strip) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const uint32_t o = T.v[c][0][r][jc];
                const uint32_t same = T.v[1 - c][0][r][jc];
                const uint32_t up = T.v[1 - c][0][r - 1][jc], dn = T.v[1 - c][0][r + 1][jc];
                // y0 is even, so y + c has the parity of r + c; colour 0
                // looks right (i + 1) on odd rows, colour 1 on even rows
                const uint32_t side = ((r + c) & 1u) ? funnel(T.v[1 - c][0][r][jc + 1], same, 1)
                                                     : funnel(same, T.v[1 - c][0][r][jc - 1], 31);
                sd_add1(o, up, dn, same, side, hist);
                np1 = bcnt_acc(o, np1);
            }
            sites += 64;
        }
        if (tb) {
            // protocol lattices (L a power of two >= 4096): every lane of the
            // strip is in it.  Lane 8 m + 7 of a DPP row gathers lanes
            // 8 m .. 8 m + 7 by three shifts within the row.
            const uint32_t x = T.v[r & 1u][0][r][jc] & 0x01010101u;
            uint32_t w = ((x | (x >> 7) | (x >> 14) | (x >> 21)) & 0xFu) << (4 * (j & 7));
            w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x111, 0xF, 0xF, true);   // row_shr:1
            w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x112, 0xF, 0xF, true);   // row_shr:2
            w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x114, 0xF, 0xF, true);   // row_shr:4
            uint32_t y = y0 + r;
            if (y >= L) y -= L;
            if ((j & 7) == 7) tb[(size_t)y * NSW + ((q0 + (uint32_t)j) >> 3)] = w;
        }
    }
}

// The residue rows of the tile's sampled rows (y = 16 b: tile rows 16, 32,
// 48, 64, as y0 is a multiple of 64): thread (plane c, row 16 (s + 1), word
// j) takes the bits t, t + 8, t + 16, t + 24 of its word for t = 0 .. 7,
// the cells 16 a + 2 t + c of the row (x = 2 i + c on even rows, i = 8 a + t),
// and merges them over 8 lanes into word (q0 + j) / 8 of residue row
// 16 b + 2 t + c, as for the T bits.  Protocol lattices only (L a power of
// two >= 4096: every lane of the strip is in it).
template <class TT>
__device__ __forceinline__ void tile_residues(const TT& T, uint32_t y0, uint32_t q0, uint32_t L,
                                              uint32_t* __restrict__ rb)
{
    const uint32_t NSW = L >> 9;
    const uint32_t c = threadIdx.x >> 7, r = 16 * (((threadIdx.x >> 5) & 3u) + 1);
    const uint32_t j = threadIdx.x & 31u;
    const uint32_t word = T.v[c][0][r][j + TT::CO];
    uint32_t y = y0 + r;
    if (y >= L) y -= L;
    uint32_t* row = rb + (size_t)y * NSW + ((q0 + j) >> 3);       // y = 16 b: residue row 16 b + rho
#pragma unroll 1
    for (uint32_t t = 0; t < 8; ++t) {
        const uint32_t x = (word >> t) & 0x01010101u;
        uint32_t w = ((x | (x >> 7) | (x >> 14) | (x >> 21)) & 0xFu) << (4 * (j & 7));
        w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x111, 0xF, 0xF, true);   // row_shr:1
        w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x112, 0xF, 0xF, true);   // row_shr:2
        w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x114, 0xF, 0xF, true);   // row_shr:4
        if ((j & 7) == 7) row[(size_t)(2 * t + c) * NSW] = w;
    }
}

// Persistent over tiles: each workgroup loads tiles (strip of kSW words by
// kTH rows, both planes, with halos) in turn and keeps its per-distance sums
// in registers; one atomic per value per workgroup at the end.  FUSED (4-bit
// Ising cells, L >= 4096): the tiles also give B, M, the counts, the sigma-h
// histogram and the T bits (tile_bmq) and the residue rows of the sampled
// rows after the T bits (tile_residues), so the B/M/Q pass need not read the
// lattice again and the sampled x pass reads packed rows; acc[14] counts the
// workgroups that saw a cell holding no spin, for which the caller runs the
// B/M/Q pass after all.
template <int MODEL, bool FUSED>
__global__ __launch_bounds__(256) void corr_short_kernel(const uint32_t* __restrict__ planes, uint32_t L, int R,
                                                         int64_t* __restrict__ Cx, int64_t* __restrict__ Cy,
                                                         int64_t* __restrict__ acc, uint32_t* __restrict__ tb)
{
    using TT = ShortTile<MODEL, FUSED>;
    __shared__ TT T;
    __shared__ int64_t red[4][66];
    __shared__ int64_t red_bmq[4][15];
    const uint32_t Wp = L >> 6;                     // tile words per row, every model
    const uint32_t nstrips = (Wp + kSW - 1) / kSW;
    const uint32_t ntiles = nstrips * (L / kTH);
    const size_t plane_units = (size_t)L * Wp;      // 16-byte vectors (4-bit) or words (1-bit) per plane
    const uint4* P4 = reinterpret_cast<const uint4*>(planes);
    // thread: word column j; waves 0 and 2 take the x axis, waves 1 and 3 the
    // y axis (uniform per wave); the two 32-lane halves of a wave and the
    // wave pair give the row group g, rows G g .. G g + G - 1 of the tile
    // (G = kTH / 4)
    const int j = threadIdx.x & (kSW - 1);
    const int wave = threadIdx.x >> 6;
    const int axis = wave & 1;
    const int g = ((wave >> 1) << 1) | ((threadIdx.x >> 5) & 1);
    int cacc[33];
#pragma unroll
    for (int k = 0; k < 33; ++k) cacc[k] = 0;
    int64_t pairs = 0;
    uint32_t bad = 0, np1 = 0, sites = 0;
    uint32_t hist[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) hist[k] = 0;
    // each workgroup takes a contiguous run of tiles, strip by strip and top
    // to bottom within a strip, so a tile's 32 halo rows are the next tile's
    // source rows: they move up in LDS and only 32 new rows are loaded
    const uint32_t RT = L / kTH;                    // row tiles per strip
    const uint32_t t_begin = (uint32_t)((uint64_t)blockIdx.x * ntiles / gridDim.x);
    const uint32_t t_end = (uint32_t)((uint64_t)(blockIdx.x + 1) * ntiles / gridDim.x);
    constexpr uint32_t NB = TT::NB;
    constexpr uint32_t COLS = TT::COLS, CO = TT::CO;
    for (uint32_t tile = t_begin; tile < t_end; ++tile) {
        const uint32_t strip = tile / RT;
        const uint32_t rt = tile - strip * RT;
        const uint32_t q0 = strip * kSW;
        const uint32_t y0 = rt * kTH;
        const bool reuse = tile != t_begin && rt != 0;
        __syncthreads();
        if (reuse) {
            // rows kTH .. kTH + kHalo - 1 become rows 0 .. kHalo - 1, one
            // (plane, bit plane) block of kTileRows x COLS words at a time
#pragma unroll
            for (uint32_t blk = 0; blk < 2 * NB; ++blk) {
                uint32_t* base = &T.v[blk / NB][blk % NB][0][0];
                for (uint32_t o = threadIdx.x; o < kHalo * COLS; o += blockDim.x)
                    base[o] = base[o + kTH * COLS];
            }
            __syncthreads();
        }
        const uint32_t row0 = reuse ? (uint32_t)kHalo : 0u;
        // the new rows: lane (column lc, row group lg) takes column lc of rows
        // row0 + lg, row0 + lg + 8, ...; then one thread per row each halo
        // column (the word right of the strip and, fused, the last cell of
        // the word left of it, periodic in the row)
        const uint32_t lc = threadIdx.x & (kSW - 1), lg = threadIdx.x >> 5;
        tile_load<MODEL>(T, planes, P4, plane_units, Wp, L, y0, row0 + lg, blockDim.x / kSW, lc + CO,
                         wrap_col(q0 + lc, Wp), bad);
        if (threadIdx.x < kTileRows - row0)
            tile_load<MODEL>(T, planes, P4, plane_units, Wp, L, y0, row0 + threadIdx.x, kTileRows, kSW + CO,
                             wrap_col(q0 + kSW, Wp), bad);
        else if (FUSED && threadIdx.x >= 128 && threadIdx.x - 128 < kTileRows - row0)
            tile_load_left(T, P4, plane_units, Wp, L, y0, row0 + threadIdx.x - 128, (q0 + Wp - 1) % Wp);
        __syncthreads();
        if (q0 + (uint32_t)j < Wp) {
            if (axis == 0) short_tile<MODEL, 0>(T, j, g, R, cacc);
            else short_tile<MODEL, 1>(T, j, g, R, cacc);
            pairs += 16 * kTH;     // kTH / 4 rows x 2 planes x 32 cells, per distance
        }
        if constexpr (FUSED) {
            tile_bmq<MODEL>(T, y0, q0, L, Wp, j, tb, hist, np1, sites);
            if (tb) tile_residues(T, y0, q0, L, tb + (size_t)L * (L >> 9));
        }
    }
    int64_t v[66];
#pragma unroll
    for (int k = 0; k < 33; ++k) {
        const int64_t sk = k > R ? 0 : (MODEL != 1 ? pairs - 2 * (int64_t)cacc[k] : (int64_t)cacc[k]);
        v[k] = axis == 0 ? sk : 0;
        v[33 + k] = axis == 1 ? sk : 0;
    }
    block_add_xy<33>(v, Cx, Cy, red);
    if (FUSED) {
        // t = 4 (two aligned neighbours) is the rest; each bond is seen from
        // both ends, so B = 2 N - sum of d over the sites (d = (8 - t) / 2)
        hist[4] = sites - hist[0] - hist[2] - hist[6] - hist[8];
        const int64_t dsum = (int64_t)hist[6] + 2 * (int64_t)hist[4] + 3 * (int64_t)hist[2] + 4 * (int64_t)hist[0];
        int64_t w[15] = {2 * (int64_t)sites - dsum, 2 * (int64_t)np1 - (int64_t)sites, (int64_t)np1,
                         (int64_t)sites - (int64_t)np1, 0};
#pragma unroll
        for (int k = 0; k < 9; ++k) w[5 + k] = (int64_t)hist[k];
        w[14] = __syncthreads_or(bad != 0) && threadIdx.x == 0 ? 1 : 0;
        block_add<15>(w, acc, red_bmq);
    }
}

// ---------------------------------------------------------------------------
// Correlations, every source, arbitrary r (full mode beyond r = 32): partners read
// from global memory.  One thread per (plane, band of rows, column), a
// chunk of up to kRChunk distances per grid row.
// ---------------------------------------------------------------------------
constexpr int kRChunk = 16;

// Word of the cells i + m .. (one word's worth, periodic in the row of W
// words), where cell i is cell 0 of word wd; wd + m / cells-per-word < 2 W.
template <int CB>
__device__ __forceinline__ uint32_t shifted_word(const uint32_t* __restrict__ row, uint32_t W, uint32_t wd, uint32_t m)
{
    const uint32_t mb = m * CB;
    const uint32_t w0 = wrap(wd + (mb >> 5), W);
    const uint32_t w1 = wrap(w0 + 1, W);
    return funnel(row[w1], row[w0], mb & 31);
}

template <int CB>
__global__ __launch_bounds__(256) void corr_all_kernel(const uint32_t* __restrict__ planes, uint32_t L, uint32_t rows,
                                                       const int32_t* __restrict__ rlist, int nr,
                                                       int64_t* __restrict__ Cx, int64_t* __restrict__ Cy)
{
    using Cl = Cell<CB>;
    const uint32_t Q = L >> Cl::kVecShift, W = L >> Cl::kWordShift;
    const int j0 = blockIdx.y * kRChunk;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t q = g % Q;
    const uint32_t rest = g / Q;
    const uint32_t nbands = L / rows;
    const uint32_t c = rest / nbands;
    const uint32_t band = rest - c * nbands;
    const size_t plane_words = (size_t)L * W;
    uint32_t xn[kRChunk], xd[kRChunk], yn[kRChunk], yd[kRChunk];
#pragma unroll
    for (int j = 0; j < kRChunk; ++j) xn[j] = xd[j] = yn[j] = yd[j] = 0;
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
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const uint32_t o = pick(v, d);
                        Cl::pair(o, pick(py, d), yn[j], yd[j]);
                        Cl::pair(o, shifted_word<CB>(prow, W, 4 * q + d, m), xn[j], xd[j]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kRChunk; ++j) {
        const int64_t sx = wave_sum((int64_t)xn[j] - 2 * (int64_t)xd[j]);
        const int64_t sy = wave_sum((int64_t)yn[j] - 2 * (int64_t)yd[j]);
        if ((threadIdx.x & 63) == 0 && j0 + j < nr) {
            atomicAdd((unsigned long long*)&Cx[j0 + j], (unsigned long long)sx);
            atomicAdd((unsigned long long*)&Cy[j0 + j], (unsigned long long)sy);
        }
    }
}

// ---------------------------------------------------------------------------
// Correlations, sampled sources (x = y = 0 mod 16), as bits.
//
// T bits: for every row y, bit j of word k of row y (plane 0) is
// [s(16 a, y) = +1] with a = 32 k + j, and for Blume-Capel plane 1 holds
// [s(16 a, y) != 0]; a row has tbits_words(L) = max(1, L / 512) words, and
// below L = 512 the NS = L / 16 bits of a row repeat to fill the word (NS
// divides 32), so a rotation by m of the word is a shift by m mod NS.  The
// site (16 a, y) has colour y & 1 and in-plane index 8 a.
//
// A sum of s s' over the pairs of two such words is, with the mask z of the
// pairs that count (both nonzero, and inside the row), popc(z) - 2
// popc(z & (a ^ b)): a product is +1 for equal signs and -1 otherwise.
// ---------------------------------------------------------------------------
template <int MODEL>
__device__ __forceinline__ int sampled_pairs(uint32_t s, uint32_t sz, uint32_t p, uint32_t pz, uint32_t valid,
                                             bool full)
{
    if (MODEL == 1) {
        const uint32_t z = sz & pz & valid;
        return (int)popc(z) - 2 * (int)popc(z & (s ^ p));
    }
    if (full) return 32 - 2 * (int)popc(s ^ p);
    return (int)popc(valid) - 2 * (int)popc(valid & (s ^ p));
}

// T bits of one row, any L: thread per output word (the bits of 32
// sources, or of NS repeated).  Used below L = 512, where the B/M/Q pass
// does not write them.
template <int MODEL>
__global__ __launch_bounds__(256) void tbits_kernel(const uint32_t* __restrict__ planes, uint32_t L,
                                                    uint32_t* __restrict__ tb)
{
    using C = Cell<MODEL == 2 ? 1 : 4>;
    const uint32_t W = L >> C::kWordShift, NS = L >> 4;
    const uint32_t NSW = L >= 512 ? L >> 9 : 1u;
    const size_t plane_words = (size_t)L * W;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < L * NSW; g += gridDim.x * blockDim.x) {
        const uint32_t y = g / NSW, k = g - y * NSW;
        const uint32_t* row = planes + (y & 1u) * plane_words + (size_t)y * W;
        uint32_t sb = 0, zb = 0;
        for (uint32_t j = 0; j < 32; ++j) {
            const int s = C::spin(row, 8u * ((32u * k + j) % NS));
            sb |= (s > 0 ? 1u : 0u) << j;
            zb |= (s != 0 ? 1u : 0u) << j;
        }
        tb[g] = sb;
        if (MODEL == 1) tb[(size_t)L * NSW + g] = zb;
    }
}

// Along x, one sampled row y = 16 b at a time (persistent over rows).  The
// row's cells go into LDS as residue rows of bits: R_rho bit a is the cell
// (16 a + rho, y).  R_0 holds the sources, and the partners of distance
// r = 16 m + rho are R_rho shifted by m: per word of 32 sources one funnel
// shift, one xor and the bit counts.  LDS holds R_0 and the residues rho0 ..
// rho0 + G - 1 (the host runs 16 / G passes when a row of all 16 residues
// does not fit), each residue row twice in a row, so the partner words
// w + m / 32 and the next need no wrap, and two words of padding after each
// row, so the rows of different residues start in different LDS banks.
// Thread k owns distance k of the launch (the host gives a launch at most
// one distance per thread): it walks every word of the row, reading the
// source words as broadcast 16-byte loads, and keeps its sum in a register
// over all the workgroup's rows; one atomic per distance and workgroup at
// the end.  Workgroups of 512 threads, several per CU, so one loads its next
// row while another works on its own.  For 4-bit Ising lattices measured with
// the fused short-distance tiles (rb set) the residue rows come ready from
// those tiles, and the row's 4-bit cells are not read at all.
//
// Building the residue rows (L >= 512): a 4-bit word w of plane c holds the
// cells x = 16 w + 2 j + c, j = 0 .. 7, i.e. bit w of residues 2 j + c, so a
// wave's 64 words give 64 bits of each of its residues by one ballot per j.
// A 1-bit word w of plane c holds x = 64 w + 2 k + c: bit k belongs to
// residue 2 (k & 7) + c at position 4 w + (k >> 3), four bits per residue,
// gathered per lane and merged over 8 lanes.
constexpr uint32_t kSxU = 4;        // row loads in flight per thread
constexpr int kSxThreads = 512;     // threads of a workgroup, and distances of a launch

__device__ __forceinline__ int sx_row(uint32_t rho, uint32_t rho0, uint32_t G)
{
    return rho - rho0 < G ? (int)(1 + rho - rho0) : -1;
}

template <int MODEL>
__global__ __launch_bounds__(kSxThreads) void corr_sxb_kernel(const uint32_t* __restrict__ planes,
                                                      const uint32_t* __restrict__ rb, uint32_t L,
                                                       const int32_t* __restrict__ rlist, int nr, uint32_t rho0,
                                                       uint32_t G, int64_t* __restrict__ Cx)
{
    constexpr int NB = MODEL == 1 ? 2 : 1;
    using C = Cell<MODEL == 2 ? 1 : 4>;
    extern __shared__ int sxb_lds[];
    uint32_t* R = reinterpret_cast<uint32_t*>(sxb_lds);   // [(1 + G) rows][NB][2 NSW], + 2 words a row
    const uint32_t W = L >> C::kWordShift, NS = L >> 4;
    const uint32_t NSW = L >= 512 ? L >> 9 : 1u;
    const uint32_t PO = 2 * NSW;                          // bit plane offset within a row
    const uint32_t rowstride = NB * PO + 2;
    const bool full = L >= 512;
    // Ising rows without invalid bits: a word's sum is 32 - 2 (differing bits)
    const bool diff_only = MODEL != 1 && full;
    const uint32_t valid = full ? 0xFFFFFFFFu : (NS >= 32 ? 0xFFFFFFFFu : ((1u << NS) - 1u));
    const size_t plane_words = (size_t)L * W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwaves = blockDim.x >> 6;
    // this thread's distance: r = 16 m + rho, the partners R_rho shifted by m
    const int k = threadIdx.x;
    const uint32_t r = k < nr ? (uint32_t)rlist[k] : 0u;
    const int rr = k < nr ? sx_row(r & 15u, rho0, G) : -1;     // -1: none, or another pass's residue
    const uint32_t m = r >> 4, sh = m & 31u;
    const uint32_t poff = (rr < 0 ? 0u : (uint32_t)rr * rowstride) + (m >> 5);
    uint32_t acc = 0;
    uint32_t rows_done = 0;
    for (uint32_t b = blockIdx.x; b < NS; b += gridDim.x) {
        const uint32_t y = 16 * b;
        ++rows_done;
        __syncthreads();
        if (MODEL == 0 && rb != nullptr) {
            // the residue rows the fused short-distance tiles wrote: row 0 the
            // sources (residue 0), rows 1 .. G the residues rho0 .., each
            // stored twice; kSxU loads in flight per thread
            const uint32_t* src = rb + (size_t)y * NSW;   // residue row 16 b + rho at src + rho NSW
            const uint32_t total = (1 + G) * NSW;
            for (uint32_t base = threadIdx.x; base < total; base += kSxU * blockDim.x) {
                uint32_t v[kSxU];
#pragma unroll
                for (uint32_t u = 0; u < kSxU; ++u) {
                    const uint32_t t = base + u * blockDim.x;
                    const uint32_t rr = t / NSW, w = t - rr * NSW;
                    const uint32_t rho = rr == 0 ? 0u : rho0 + rr - 1;
                    v[u] = t < total ? src[(size_t)rho * NSW + w] : 0u;
                }
#pragma unroll
                for (uint32_t u = 0; u < kSxU; ++u) {
                    const uint32_t t = base + u * blockDim.x;
                    if (t < total) {
                        const uint32_t rr = t / NSW, w = t - rr * NSW;
                        R[rr * rowstride + w] = v[u];
                        R[rr * rowstride + NSW + w] = v[u];
                    }
                }
            }
        } else if (L < 512) {
            // one word per residue row, its NS bits repeated
            for (uint32_t t = threadIdx.x; t < (1 + G) * NB; t += blockDim.x) {
                const uint32_t rr = t / NB, plane = t - rr * NB;
                const uint32_t rho = rr == 0 ? 0u : rho0 + rr - 1;
                const uint32_t c = rho & 1u;                     // (x + y) & 1 with y even
                const uint32_t* row = planes + c * plane_words + (size_t)y * W;
                uint32_t v = 0;
                for (uint32_t j = 0; j < 32; ++j) {
                    const int s = C::spin(row, (16u * (j % NS) + rho) >> 1);
                    v |= ((plane == 0 ? s > 0 : s != 0) ? 1u : 0u) << j;
                }
                R[rr * rowstride + plane * PO] = v;
            }
        } else if (C::kPerWord == 8) {
            // a wave takes 64 consecutive words of the row at a time (2 W of
            // them, both planes; W is a multiple of 32, so a group of 64 is
            // whole): the bookkeeping is per wave.  The loads of kSxU groups
            // are issued together, so a wave waits for memory once per kSxU
            // groups rather than once per group.
            const uint32_t step = 64u * (uint32_t)nwaves;
            for (uint32_t base = __builtin_amdgcn_readfirstlane(64u * (uint32_t)wave); base < 2 * W;
                 base += kSxU * step) {
                uint32_t words[kSxU];
#pragma unroll
                for (uint32_t u = 0; u < kSxU; ++u) {
                    const uint32_t idx = base + u * step + (uint32_t)lane;
                    const uint32_t c = idx >= W ? 1u : 0u;
                    words[u] = idx < 2 * W ? planes[c * plane_words + (size_t)y * W + (idx - c * W)] : 0u;
                }
#pragma unroll
                for (uint32_t u = 0; u < kSxU; ++u) {
                    const uint32_t idx0 = base + u * step;
                    if (idx0 >= 2 * W) break;
                    const uint32_t word = words[u];
                    // lanes 0..31 and 32..63 cover 32 words each, of one plane each
                    const uint32_t c_lo = idx0 >= W ? 1u : 0u, c_hi = idx0 + 32 >= W ? 1u : 0u;
                    const uint32_t k_lo = (idx0 - c_lo * W) >> 5, k_hi = (idx0 + 32 - c_hi * W) >> 5;
                    uint64_t ms[8], mz[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        ms[j] = __ballot((word >> (4 * j + 1)) & 1u);
                        mz[j] = NB == 2 ? __ballot(((~word) >> (4 * j)) & 1u) : 0u;
                    }
                    if (c_lo == c_hi) {
                        // L >= 1024: the two halves are words k_lo, k_lo + 1 (k_lo
                        // even) of one residue row, 8-byte aligned in LDS
                        if (lane == 0) {
#pragma unroll
                            for (int j = 0; j < 8; ++j) {
                                const uint32_t t = 2u * j + c_lo - rho0;       // the residue's slot - 1
                                if (t < G) {
                                    uint32_t* dst = R + (1 + t) * rowstride + k_lo;
                                    *reinterpret_cast<uint2*>(dst) = make_uint2((uint32_t)ms[j], (uint32_t)(ms[j] >> 32));
                                    if (NB == 2)
                                        *reinterpret_cast<uint2*>(dst + PO) =
                                            make_uint2((uint32_t)mz[j], (uint32_t)(mz[j] >> 32));
                                }
                            }
                            if (c_lo == 0) {                                   // residue 0: the sources
                                *reinterpret_cast<uint2*>(R + k_lo) = make_uint2((uint32_t)ms[0], (uint32_t)(ms[0] >> 32));
                                if (NB == 2)
                                    *reinterpret_cast<uint2*>(R + PO + k_lo) =
                                        make_uint2((uint32_t)mz[0], (uint32_t)(mz[0] >> 32));
                            }
                        }
                        continue;
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        if (lane == 0) {
                            const uint32_t rl_lo = 2 * j + c_lo, rl_hi = 2 * j + c_hi;
                            const int r_lo = sx_row(rl_lo, rho0, G), r_hi = sx_row(rl_hi, rho0, G);
                            if (r_lo >= 0) {
                                R[r_lo * rowstride + k_lo] = (uint32_t)ms[j];
                                if (NB == 2) R[r_lo * rowstride + PO + k_lo] = (uint32_t)mz[j];
                            }
                            if (r_hi >= 0) {
                                R[r_hi * rowstride + k_hi] = (uint32_t)(ms[j] >> 32);
                                if (NB == 2) R[r_hi * rowstride + PO + k_hi] = (uint32_t)(mz[j] >> 32);
                            }
                            if (rl_lo == 0) {                            // the sources
                                R[k_lo] = (uint32_t)ms[j];
                                if (NB == 2) R[PO + k_lo] = (uint32_t)mz[j];
                            }
                            if (rl_hi == 0) {
                                R[k_hi] = (uint32_t)(ms[j] >> 32);
                                if (NB == 2) R[PO + k_hi] = (uint32_t)(mz[j] >> 32);
                            }
                        }
                    }
                }
            }
        } else {
            // as above, the loads of kSxU words per thread issued together
            for (uint32_t base = threadIdx.x; base < 2 * W; base += kSxU * blockDim.x) {
                uint32_t words[kSxU];
#pragma unroll
                for (uint32_t u = 0; u < kSxU; ++u) {
                    const uint32_t idx = base + u * blockDim.x;
                    const uint32_t c = idx >= W ? 1u : 0u;
                    words[u] = idx < 2 * W ? planes[c * plane_words + (size_t)y * W + (idx - c * W)] : 0u;
                }
#pragma unroll
                for (uint32_t u = 0; u < kSxU; ++u) {
                    const uint32_t idx = base + u * blockDim.x;
                    if (idx >= 2 * W) break;
                    const uint32_t c = idx >= W ? 1u : 0u;
                    const uint32_t w = idx - c * W;
                    const uint32_t word = words[u];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const uint32_t x = (word >> j) & 0x01010101u;     // bits j, j + 8, j + 16, j + 24
                        const uint32_t nib = (x | (x >> 7) | (x >> 14) | (x >> 21)) & 0xFu;
                        uint32_t v = nib << (4u * (w & 7u));
                        v |= __shfl_xor(v, 1);
                        v |= __shfl_xor(v, 2);
                        v |= __shfl_xor(v, 4);
                        if ((w & 7u) == 0) {
                            const uint32_t rho = 2 * j + c;
                            const int rr = sx_row(rho, rho0, G);
                            if (rr >= 0) R[rr * rowstride + (w >> 3)] = v;
                            if (rho == 0) R[w >> 3] = v;
                        }
                    }
                }
            }
        }
        __syncthreads();
        // the second copy of each residue row (the packed rows come with it)
        for (uint32_t t = threadIdx.x; !(MODEL == 0 && rb != nullptr) && t < G * NB * NSW; t += blockDim.x) {
            const uint32_t rr = 1 + t / (NB * NSW), rest = t % (NB * NSW);
            const uint32_t pl = rest / NSW, w = rest - pl * NSW;
            uint32_t* row = R + rr * rowstride + pl * PO;
            row[NSW + w] = row[w];
        }
        __syncthreads();
        if (rr >= 0) {
            const uint32_t* P = R + poff;
            if (diff_only && (NSW & 3u) == 0) {
                for (uint32_t w = 0; w < NSW; w += 4) {
                    const uint4 s4 = *reinterpret_cast<const uint4*>(R + w);
                    const uint32_t p0 = P[w], p1 = P[w + 1], p2 = P[w + 2], p3 = P[w + 3], p4 = P[w + 4];
                    acc = bcnt_acc(s4.x ^ funnel(p1, p0, sh), acc);
                    acc = bcnt_acc(s4.y ^ funnel(p2, p1, sh), acc);
                    acc = bcnt_acc(s4.z ^ funnel(p3, p2, sh), acc);
                    acc = bcnt_acc(s4.w ^ funnel(p4, p3, sh), acc);
                }
            } else {
                for (uint32_t w = 0; w < NSW; ++w) {
                    const uint32_t p = funnel(P[w + 1], P[w], sh);
                    if (diff_only) {
                        acc = bcnt_acc(R[w] ^ p, acc);
                    } else {
                        uint32_t sz = 0, pz = 0;
                        if (NB == 2) {
                            sz = R[PO + w];
                            pz = funnel(P[PO + w + 1], P[PO + w], sh);
                        }
                        acc += (uint32_t)sampled_pairs<MODEL>(R[w], sz, p, pz, valid, full);
                    }
                }
            }
        }
    }
    // Ising from L = 512 on: the sum counts differing bits (32 pairs a word)
    if (rr >= 0) {
        const int64_t v = diff_only ? 32 * (int64_t)NSW * rows_done - 2 * (int64_t)acc : (int64_t)(int32_t)acc;
        if (v != 0) atomicAdd((unsigned long long*)&Cx[k], (unsigned long long)v);
    }
}

// Along y: S_y(r) = sum over the sampled rows b and words k of the pairs of
// T row 16 b and T row 16 b + r (mod L).  Thread per (source row, group of
// WPT words: 4 from L = 2048 on, read as one 16-byte load), grid row per
// chunk of 32 distances; a thread keeps the source words and the 32
// distance sums in registers, the target words come from L2.  Ising rows
// from L = 512 on have no invalid bits: the sum is then 32 per word minus
// twice the count of differing bits, which is all the loop counts.
constexpr int kYChunk = 32;

template <int WPT>
__device__ __forceinline__ void load_words(const uint32_t* __restrict__ p, uint32_t (&w)[WPT])
{
    if (WPT == 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        w[0] = v.x;
        w[WPT > 1 ? 1 : 0] = v.y;
        w[WPT > 2 ? 2 : 0] = v.z;
        w[WPT > 3 ? 3 : 0] = v.w;
    } else {
#pragma unroll
        for (int i = 0; i < WPT; ++i) w[i] = p[i];
    }
}

template <int MODEL, int WPT>
__global__ __launch_bounds__(256) void corr_syb_kernel(const uint32_t* __restrict__ tb, uint32_t L,
                                                       const int32_t* __restrict__ rlist, int nr,
                                                       int64_t* __restrict__ Cy)
{
    constexpr int NB = MODEL == 1 ? 2 : 1;
    const uint32_t NS = L >> 4;
    const uint32_t NSW = L >= 512 ? L >> 9 : 1u;
    const uint32_t groups = NSW / WPT;                    // a power of two
    const uint32_t g_log = 31 - __builtin_clz(groups);
    const bool full = L >= 512;
    const bool diff_only = MODEL != 1 && full;
    const uint32_t valid = full ? 0xFFFFFFFFu : (NS >= 32 ? 0xFFFFFFFFu : ((1u << NS) - 1u));
    const size_t zoff = (size_t)L * NSW;                  // plane 1 (Blume-Capel nonzero bits)
    const int k0 = blockIdx.y * kYChunk;
    const int kn = min(kYChunk, nr - k0);
    uint32_t rr[kYChunk];
    int acc[kYChunk];
#pragma unroll
    for (int k = 0; k < kYChunk; ++k) {
        rr[k] = k < kn ? (uint32_t)rlist[k0 + k] : 0u;
        acc[k] = 0;
    }
    int words = 0;                                        // source words taken by this thread
    const uint32_t pairs = NS * groups;
    // workgroup ids go round-robin to the 8 XCDs: XCD x takes the x-th eighth
    // of the source rows, so neighbouring source rows (whose partner rows at
    // nearby distances coincide) meet in the same L2
    const uint32_t nb = gridDim.x;
    const uint32_t bx = (nb & 7u) == 0 ? (blockIdx.x & 7u) * (nb >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    for (uint32_t p = bx * blockDim.x + threadIdx.x; p < pairs; p += gridDim.x * blockDim.x) {
        const uint32_t b = p >> g_log, w = (p & (groups - 1)) * WPT;
        const uint32_t y = 16 * b;
        uint32_t s[WPT], sz[WPT];
        load_words<WPT>(tb + (size_t)y * NSW + w, s);
        if (NB == 2) load_words<WPT>(tb + zoff + (size_t)y * NSW + w, sz);
        words += WPT;
#pragma unroll
        for (int k = 0; k < kYChunk; ++k) {
            if (k < kn) {
                const uint32_t yp = (y + rr[k]) & (L - 1);
                uint32_t t[WPT], tz[WPT];
                load_words<WPT>(tb + (size_t)yp * NSW + w, t);
                if (NB == 2) load_words<WPT>(tb + zoff + (size_t)yp * NSW + w, tz);
#pragma unroll
                for (int i = 0; i < WPT; ++i) {
                    if (diff_only)
                        acc[k] += (int)popc(s[i] ^ t[i]);
                    else
                        acc[k] += sampled_pairs<MODEL>(s[i], NB == 2 ? sz[i] : 0u, t[i], NB == 2 ? tz[i] : 0u, valid,
                                                       full);
                }
            }
        }
    }
    __shared__ int red[4][kYChunk];
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kYChunk; ++k) {
        const int v = diff_only ? 32 * words - 2 * acc[k] : acc[k];
        const int s2 = wave_sum_i32(v);
        if ((threadIdx.x & 63) == 0) red[wave][k] = s2;
    }
    __syncthreads();
    if ((int)threadIdx.x < kn) {
        const int k = threadIdx.x;
        const int64_t tot = (int64_t)red[0][k] + red[1][k] + red[2][k] + red[3][k];
        if (tot != 0) atomicAdd((unsigned long long*)&Cy[k0 + k], (unsigned long long)tot);
    }
}

// Along y, the sampled distances r0 .. r0 + nl - 1 that follow one another
// (the protocol's linear range).  Source rows 16 b and 16 (b + 1) meet the
// same partner rows at distances r + 16 and r, so a workgroup takes a band of
// kYLRows source rows and stages their partner rows, 16 (kYLRows - 1) +
// kYLDist consecutive T rows, in LDS, kYLWords words of each at a time (a
// row of T words is a multiple of 8 from L = 4096 on; rows padded by one
// vector); thread d owns distance r0 + kYLDist c + d (c the grid
// row) and keeps its count in a register over the band and all columns.
// Ising rows from L = 4096 on: no invalid bits, so a word's sum is 32 minus
// twice its differing bits.
constexpr int kYLRows = 16;
constexpr int kYLDist = 256;
constexpr int kYLWords = 8;
constexpr int kYLVec = kYLWords / 4;                  // 16-byte vectors of a row's column
constexpr int kYLTgt = 16 * (kYLRows - 1) + kYLDist;
constexpr int kYLPad = kYLVec + 1;                    // 16-byte vectors per staged row

__global__ __launch_bounds__(256) void corr_sylin_kernel(const uint32_t* __restrict__ tb, uint32_t L, uint32_t r0,
                                                         int nl, int64_t* __restrict__ Cy)
{
    __shared__ uint4 tgt[kYLTgt * kYLPad];
    __shared__ uint4 src[kYLRows * kYLVec];
    const uint32_t NSW = L >> 9;
    // bands in XCD-contiguous eighths (workgroup ids go round-robin to the
    // XCDs), so neighbouring bands share their partner rows in one L2
    const uint32_t nb = gridDim.x;
    const uint32_t band = (nb & 7u) == 0 ? (blockIdx.x & 7u) * (nb >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    const uint32_t b0 = band * kYLRows;
    const int c = blockIdx.y;
    const uint32_t ra = r0 + (uint32_t)c * kYLDist;
    const int nd = min(kYLDist, nl - c * kYLDist);
    const uint32_t nvec = (16 * (kYLRows - 1) + (uint32_t)nd) * kYLVec;
    const int d = threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t w0 = 0; w0 < NSW; w0 += kYLWords) {
        __syncthreads();
        // vector v: row v / kYLVec, words w0 + 4 (v % kYLVec) ..; 8 loads in flight
        for (uint32_t base = threadIdx.x; base < nvec; base += 8 * blockDim.x) {
            uint4 x[8];
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) {
                const uint32_t v = base + u * blockDim.x;
                const uint32_t y = (16 * b0 + ra + v / kYLVec) & (L - 1);
                x[u] = v < nvec ? *reinterpret_cast<const uint4*>(tb + (size_t)y * NSW + w0 + 4 * (v % kYLVec))
                                : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) {
                const uint32_t v = base + u * blockDim.x;
                if (v < nvec) tgt[(v / kYLVec) * kYLPad + v % kYLVec] = x[u];
            }
        }
        if (threadIdx.x < kYLRows * kYLVec) {
            const uint32_t i = threadIdx.x / kYLVec, j = threadIdx.x % kYLVec;
            src[threadIdx.x] = *reinterpret_cast<const uint4*>(tb + (size_t)(16 * (b0 + i)) * NSW + w0 + 4 * j);
        }
        __syncthreads();
        if (d < nd) {
            for (int i = 0; i < kYLRows; ++i) {
#pragma unroll
                for (int j = 0; j < kYLVec; ++j) {
                    const uint4 a = src[i * kYLVec + j], t = tgt[(16 * i + d) * kYLPad + j];
                    acc = bcnt_acc(a.x ^ t.x, acc);
                    acc = bcnt_acc(a.y ^ t.y, acc);
                    acc = bcnt_acc(a.z ^ t.z, acc);
                    acc = bcnt_acc(a.w ^ t.w, acc);
                }
            }
        }
    }
    if (d < nd) {
        const int64_t v = (int64_t)32 * kYLRows * NSW - 2 * (int64_t)acc;
        atomicAdd((unsigned long long*)&Cy[c * kYLDist + d], (unsigned long long)v);
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

// Optional cap on the workgroups of the persistent measurement kernels
// (B/M/Q pass, short-distance tiles, sampled x rows): the environment
// variable MCL_MEASURE_GRID, read at every launch.  It changes how the work
// is split over workgroups, never the sums; a test uses it to give each
// workgroup several tasks, tiles and rows at small L.
uint32_t grid_cap(uint32_t want)
{
    if (const char* e = std::getenv("MCL_MEASURE_GRID")) {
        const long long v = std::atoll(e);
        if (v > 0 && (uint64_t)v < want) return (uint32_t)v;
    }
    return want;
}

// Optional band height of the B/M/Q pass: MCL_MEASURE_ROWS (2 to 64, read
// at every launch; the largest divisor of L up to it is taken).  Like the
// grid cap it changes the split of the work only; a test uses it to run the
// 64-row bands of large lattices at small L.
int64_t bmq_rows(const Geom& g)
{
    if (const char* e = std::getenv("MCL_MEASURE_ROWS")) {
        const long long v = std::atoll(e);
        if (v >= 2 && v <= 64) return pick_rows(g.L, v);
    }
    return pick_rows(g.L, g.Q * (g.L / 64) >= (int64_t(1) << 20) ? 64 : 32);
}

hipError_t launch_bmq(const Geom& g, int model, int64_t* acc, uint32_t* tbits, hipStream_t s)
{
    // one thread per task, bands of 64 rows while that leaves 2^20 tasks or
    // more (else 32).  The words beside a vector come from the neighbouring
    // lanes, so the lines a pass reads twice are the halo rows of its bands
    // and those at workgroup edges.  Measured at L = 2^17 (4-bit Ising),
    // bytes read against the lattice's: 1.50x with every halo word loaded
    // from memory, 1.12x with lane exchanges, 1.09x with the XCD-aware
    // workgroup order as well, 1.056x with 64-row bands (16 rows: 1.15x);
    // 2.06 - 2.09 ms each way once the halo loads were gone.
    const int64_t rows = bmq_rows(g);
    const int64_t threads = g.Q * (g.L / rows);
    const uint32_t grid = grid_cap((uint32_t)((threads + 255) / 256));
    const uint32_t L = (uint32_t)g.L, R = (uint32_t)rows;
    // the pass writes the T bits from L = 512 on; below, a kernel of its own
    uint32_t* tb = g.L >= 512 ? tbits : nullptr;
    const bool wave_rows = (g.Q & 63) == 0;
    if (model == 2) {
        if (wave_rows)
            hipLaunchKernelGGL((bmq_kernel<2, true>), dim3(grid), dim3(256), 0, s, g.plane(0), g.plane(1), L, R, acc, tb);
        else
            hipLaunchKernelGGL((bmq_kernel<2, false>), dim3(grid), dim3(256), 0, s, g.plane(0), g.plane(1), L, R, acc, tb);
    } else if (model == 1) {
        if (wave_rows)
            hipLaunchKernelGGL((bmq_kernel<1, true>), dim3(grid), dim3(256), 0, s, g.plane(0), g.plane(1), L, R, acc, tb);
        else
            hipLaunchKernelGGL((bmq_kernel<1, false>), dim3(grid), dim3(256), 0, s, g.plane(0), g.plane(1), L, R, acc, tb);
    } else {
        if (wave_rows)
            hipLaunchKernelGGL((bmq_kernel<0, true>), dim3(grid), dim3(256), 0, s, g.plane(0), g.plane(1), L, R, acc, tb);
        else
            hipLaunchKernelGGL((bmq_kernel<0, false>), dim3(grid), dim3(256), 0, s, g.plane(0), g.plane(1), L, R, acc, tb);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !tbits || tb) return e;
    const uint32_t nw = (uint32_t)(g.L * tbits_words(g.L));
    const dim3 tg((nw + 255) / 256);
    if (model == 2)
        hipLaunchKernelGGL(tbits_kernel<2>, tg, dim3(256), 0, s, g.plane0, L, tbits);
    else if (model == 1)
        hipLaunchKernelGGL(tbits_kernel<1>, tg, dim3(256), 0, s, g.plane0, L, tbits);
    else
        hipLaunchKernelGGL(tbits_kernel<0>, tg, dim3(256), 0, s, g.plane0, L, tbits);
    return hipGetLastError();
}

bool bmq_fused(const Geom& g, int model)
{
    if (model != 0 || g.L < 4096) return false;
    if (const char* e = std::getenv("MCL_MEASURE_FUSED")) return std::atoi(e) != 0;
    return true;
}

hipError_t launch_corr_short(const Geom& g, int model, int R, int64_t* Cx, int64_t* Cy, int64_t* acc,
                             uint32_t* tbits, hipStream_t s)
{
    if (R < 0) return hipSuccess;
    const uint32_t Wp = (uint32_t)(g.L >> 6);
    const uint32_t nstrips = (Wp + kSW - 1) / kSW;
    const uint32_t ntiles = nstrips * (uint32_t)(g.L / kTH);
    const dim3 grid(grid_cap(std::min<uint32_t>(ntiles, 1024)));
    const uint32_t L = (uint32_t)g.L;
    if (acc && (model != 0 || g.L < 4096 || (tbits && (Wp % kSW) != 0))) return hipErrorInvalidValue;
    if (acc) {
        hipLaunchKernelGGL((corr_short_kernel<0, true>), grid, dim3(256), 0, s, g.plane0, L, R, Cx, Cy, acc, tbits);
    } else if (model == 0) {
        hipLaunchKernelGGL((corr_short_kernel<0, false>), grid, dim3(256), 0, s, g.plane0, L, R, Cx, Cy, acc, tbits);
    } else if (model == 1) {
        hipLaunchKernelGGL((corr_short_kernel<1, false>), grid, dim3(256), 0, s, g.plane0, L, R, Cx, Cy, acc, tbits);
    } else {
        hipLaunchKernelGGL((corr_short_kernel<2, false>), grid, dim3(256), 0, s, g.plane0, L, R, Cx, Cy, acc, tbits);
    }
    return hipGetLastError();
}

hipError_t launch_corr_all(const Geom& g, const int32_t* r_dev, int nr, int64_t* Cx, int64_t* Cy, hipStream_t s)
{
    if (nr <= 0) return hipSuccess;
    const int64_t rows = pick_rows(g.L, 16);
    const int64_t threads = 2 * g.Q * (g.L / rows);
    const uint32_t chunks = (uint32_t)((nr + kRChunk - 1) / kRChunk);
    const dim3 grid((uint32_t)((threads + 255) / 256), chunks);
    if (g.cb == 1)
        hipLaunchKernelGGL(corr_all_kernel<1>, grid, dim3(256), 0, s, g.plane0, (uint32_t)g.L, (uint32_t)rows, r_dev,
                           nr, Cx, Cy);
    else
        hipLaunchKernelGGL(corr_all_kernel<4>, grid, dim3(256), 0, s, g.plane0, (uint32_t)g.L, (uint32_t)rows, r_dev,
                           nr, Cx, Cy);
    return hipGetLastError();
}

namespace {

// LDS bytes the x-correlation kernel may use: 160 KiB, or less when the
// environment variable MCL_SX_LDS_BUDGET says so (a test uses it to run the
// multi-pass form at small L).
size_t sx_lds_budget()
{
    size_t budget = 160u * 1024u;
    if (const char* e = std::getenv("MCL_SX_LDS_BUDGET")) {
        const long long v = std::atoll(e);
        if (v > 0 && (size_t)v < budget) budget = (size_t)v;
    }
    return budget;
}

template <int MODEL>
hipError_t corr_sampled_x(const Geom& g, const SampledArgs& a, hipStream_t s)
{
    const uint32_t L = (uint32_t)g.L, NS = L / 16;
    if ((L & (L - 1)) != 0 || L < 64) return hipErrorInvalidValue;   // the protocol's lattices only
    if (a.rbits && (MODEL != 0 || L < 4096)) return hipErrorInvalidValue;
    constexpr int NB = MODEL == 1 ? 2 : 1;
    // along x: LDS holds the source row and G residue rows of bits, each
    // row stored twice and padded by two words; a launch takes one distance
    // per thread
    const size_t rowb = ((size_t)NB * 2 * tbits_words(L) + 2) * 4, budget = sx_lds_budget();
    const uint32_t gx = grid_cap(std::min<uint32_t>(NS, 1024));
    uint32_t G = 16;
    while (G > 1 && rowb * (1 + G) > budget) G >>= 1;
    if (rowb * (1 + G) > budget) return hipErrorInvalidValue;
    const int max_r = kSxThreads;
    hipError_t e = hipSuccess;
    for (int j0 = 0; j0 < a.nr; j0 += max_r) {
        const int nr = std::min(max_r, a.nr - j0);
        const size_t lds = rowb * (1 + G);
        // the attribute belongs to the current device: set it for every launch that needs it
        if (lds > 64u * 1024u) {
            e = hipFuncSetAttribute((const void*)corr_sxb_kernel<MODEL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds);
            if (e != hipSuccess) return e;
        }
        for (uint32_t rho0 = 0; rho0 < 16; rho0 += G) {
            hipLaunchKernelGGL((corr_sxb_kernel<MODEL>), dim3(gx), dim3(kSxThreads), lds, s, g.plane0, a.rbits, L, a.r + j0, nr, rho0,
                               G, a.Cx + j0);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template <int MODEL>
hipError_t corr_sampled_y(const Geom& g, const SampledArgs& a, hipStream_t sy)
{
    const uint32_t L = (uint32_t)g.L, NS = L / 16;
    if ((L & (L - 1)) != 0 || L < 64) return hipErrorInvalidValue;
    // the consecutive distances first, for Ising from L = 4096 on: partner
    // rows staged in LDS per band of source rows
    int done = 0;
    if (MODEL != 1 && L >= 4096 && a.nlin > 0) {
        const dim3 gl(NS / kYLRows, (uint32_t)((a.nlin + kYLDist - 1) / kYLDist));
        hipLaunchKernelGGL(corr_sylin_kernel, gl, dim3(kYLDist), 0, sy, a.tbits, L, a.rlin0, a.nlin, a.Cy);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        done = a.nlin;
    }
    const int nr = a.nr - done;
    if (nr <= 0) return hipSuccess;
    // the others: a group of 4 source-row words per thread from L = 2048 on
    // (one word below), a grid row per 32 distances
    const uint32_t wpt = tbits_words(L) >= 4 ? 4u : 1u;
    const uint64_t groups = (uint64_t)NS * (tbits_words(L) / wpt);
    const uint32_t gyx = grid_cap((uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((groups + 255) / 256, 2048)));
    const dim3 gy(gyx, (uint32_t)((nr + kYChunk - 1) / kYChunk));
    if (wpt == 4)
        hipLaunchKernelGGL((corr_syb_kernel<MODEL, 4>), gy, dim3(256), 0, sy, a.tbits, L, a.r + done, nr, a.Cy + done);
    else
        hipLaunchKernelGGL((corr_syb_kernel<MODEL, 1>), gy, dim3(256), 0, sy, a.tbits, L, a.r + done, nr, a.Cy + done);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_corr_sampled_x(const Geom& g, int model, const SampledArgs& a, hipStream_t s)
{
    if (a.nr <= 0) return hipSuccess;
    return model == 2 ? corr_sampled_x<2>(g, a, s) : model == 1 ? corr_sampled_x<1>(g, a, s) : corr_sampled_x<0>(g, a, s);
}

hipError_t launch_corr_sampled_y(const Geom& g, int model, const SampledArgs& a, hipStream_t s)
{
    if (a.nr <= 0) return hipSuccess;
    return model == 2 ? corr_sampled_y<2>(g, a, s) : model == 1 ? corr_sampled_y<1>(g, a, s) : corr_sampled_y<0>(g, a, s);
}

}  // namespace mcl
