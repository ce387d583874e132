// Device code of the half-sweep shared by the one-lattice kernel and the
// batched kernel: acceptance masks, the Ising and Blume-Capel vector
// updates and the walk of one thread down a band of rows (Ising and Blume-Capel).
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
#pragma once

#include "common.h"

namespace mcl {
namespace dev {

__device__ __forceinline__ uint32_t lo32(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }

// High word of a Philox counter: 0 while every block index of the lattice
// fits 32 bits (HM 0); the wave-uniform value hu when the caller has shown
// that all of the wave's blocks share it (HM 1, kept in a scalar register);
// else per lane (HM 2).
template <int HM>
__device__ __forceinline__ uint32_t hiw(uint64_t b, uint32_t hu)
{
    return HM == 0 ? 0u : (HM == 1 ? hu : hi32(b));
}

__device__ __forceinline__ uint32_t pick(const uint4& v, int d)
{
    return d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w;
}

// ---------------------------------------------------------------------------
// Acceptance bits of the 32 cells of one 16-byte vector.  Cell j (0..7) of
// word d (0..3) is in-colour site kv + 8d + j; its accept draw is output
// word j & 3 of Philox block (kv >> 2) + 2d + (j >> 2).  Returns, for each
// threshold T, a 32-bit mask whose bit 4j + d is [u < T]: the "transposed"
// order lets each mask be built with one carry-chain add per cell
// (acc = acc + acc + carry) and lets word d read its cells' bits at nibble
// bit 0 as (mask >> d) & 0x11111111.
// ---------------------------------------------------------------------------
// The block index is cb + blk0 + k (k = 0..7) with cb wave-uniform (0 on
// the per-lane walk).
template <int HM>
__device__ __forceinline__ void accept_masks(uint64_t blk0, uint32_t cb, uint32_t t, uint32_t color, uint32_t k0,
                                             uint32_t k1, uint32_t hu, uint32_t T4, uint32_t T8, uint32_t& m4,
                                             uint32_t& m8)
{
    uint32_t a4 = 0, a8 = 0;
    // the low counter words of the vector's 8 blocks are cb + lo32(blk0) + k
    // without a wrap unless the high word varies per lane (HM 2), so the first
    // round's product M0 (cb + lo32(blk0) + k) is one multiply-add with the
    // uniform addend M0 cb + M0 k
    const uint32_t c0 = lo32(blk0);
    const uint64_t mb = (uint64_t)kPhiloxM0 * cb;
#pragma unroll
    for (int h = 1; h >= 0; --h) {
        Philox4 P[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint64_t b = blk0 + 2 * d + h;
            if (HM == 2)
                P[d] = philox4x32_10(lo32(b), hiw<HM>(b, hu), t, color, k0, k1);
            else
                P[d] = philox4x32_10_p0(mad_m0(c0, mb + (uint64_t)kPhiloxM0 * (uint32_t)(2 * d + h)),
                                        hiw<HM>(b, hu), t, color, k0, k1);
        }
#pragma unroll
        for (int jj = 3; jj >= 0; --jj)
#pragma unroll
            for (int d = 3; d >= 0; --d) {
                const uint32_t u = philox_word(P[d], jj);
                a4 = shift_in_lt(a4, u, T4);
                a8 = shift_in_lt(a8, u, T8);
            }
    }
    m4 = a4;
    m8 = a8;
}

// Horizontal neighbour word of word d of vector `mid`: cells i - 1 (even
// row parity) or i + 1 (odd) of the other plane, with `halo` the adjacent
// word outside the vector on that side.
__device__ __forceinline__ uint32_t horizontal(const uint4& mid, int d, uint32_t halo, bool odd)
{
    const uint32_t w = pick(mid, d);
    if (odd) return funnel(d < 3 ? pick(mid, d + 1) : halo, w, 4);
    return funnel(w, d > 0 ? pick(mid, d - 1) : halo, 28);
}

// ---------------------------------------------------------------------------
// Ising vector update (32 cells).  Cells hold n in {0, 2}; n ^ src is 2
// for a misaligned neighbour, so S = 4 + the per-nibble sum of the four
// xors is 4 + 2 m, m the number of misaligned neighbours (at most 12: no
// carry between nibbles).  The flip rule of section 3.2 (always with at most
// two aligned neighbours, with probability e^{-4 beta} with three,
// e^{-8 beta} with four) reads, with a4 = [u < T4] and a8 = [u < T8], which
// implies a4 since T8 <= T4:
//   flip = [m >= 2] | ([m == 1] & a4) | ([m == 0] & a8)
//        = S.bit3 | (S.bit1 & a4) | a8,
// since m >= 2 iff S >= 8, and for m < 2 bit 1 of S is [m == 1].  Every
// term is moved to nibble bit 1, where a flip toggles n (0 <-> 2): bit 3 by
// a shift of S, and a4 / a8 by shifting the transposed masks so that bit
// 4j + d (cell j of word d) lands on 4j + 1.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ uint32_t to_bit1(uint32_t m)
{
    return D == 0 ? (m << 1) : (m >> (D - 1));
}

template <int HM>
__device__ __forceinline__ uint4 ising_vec(const uint4& src, const uint4& up, const uint4& dn, const uint4& mid,
                                           uint32_t halo, bool odd, uint64_t blk0, uint32_t cb, uint32_t t,
                                           uint32_t color, uint32_t k0, uint32_t k1, uint32_t hu, uint32_t T4,
                                           uint32_t T8)
{
    uint32_t m4, m8;
    accept_masks<HM>(blk0, cb, t, color, k0, k1, hu, T4, T8, m4, m8);
    uint32_t res[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t s = pick(src, d);
        const uint32_t hs = horizontal(mid, d, halo, odd);
        uint32_t S = xad(pick(up, d), s, 0x44444444u);
        S = xad(pick(dn, d), s, S);
        S = xad(pick(mid, d), s, S);
        S = xad(hs, s, S);
        const uint32_t a4 = d == 0 ? to_bit1<0>(m4) : d == 1 ? to_bit1<1>(m4) : d == 2 ? to_bit1<2>(m4) : to_bit1<3>(m4);
        const uint32_t a8 = d == 0 ? to_bit1<0>(m8) : d == 1 ? to_bit1<1>(m8) : d == 2 ? to_bit1<2>(m8) : to_bit1<3>(m8);
        const uint32_t f = ((S >> 2) | (S & a4) | a8) & 0x22222222u;
        res[d] = s ^ f;
    }
    return make_uint4(res[0], res[1], res[2], res[3]);
}

// ---------------------------------------------------------------------------
// Blume-Capel vector update (32 cells).  Per cell: the proposal
// s' = ((n + 1 + b) mod 3) - 1 (n = s + 1, b the proposal bit), then a table
// lookup on (n, b, sum of neighbour cells) gives E = thr, or 2^32 where
// dE <= 0, and accept = [u < E].  Word-level: n + 1 + b and its reduction
// mod 3 are nibble-parallel, the table index of each cell is a byte built
// for 4 cells at a time, and the accept bits gate the new values in with a
// bit select.
// ---------------------------------------------------------------------------
// Spread the low 8 bits of x to bit 0 of the 8 nibbles.
__device__ __forceinline__ uint32_t spread8(uint32_t x)
{
    x &= 0xFFu;
    x = shl_or<12>(x, x) & 0x000F000Fu;
    x = shl_or<6>(x, x) & 0x03030303u;
    x = shl_or<3>(x, x) & 0x11111111u;
    return x;
}

// LDS table: entry (key << 4) | sum, key = 2 n + b, holds A = -E as a
// 64-bit value (x = low word, y = high word), so that the high word of
// u + A is -[u < E].  256 entries: every byte a corrupted cell could form
// stays in bounds (entries that no spin state reaches reject).
struct BCLds {
    uint2 e[256];
};

__device__ __forceinline__ uint2 bc_addend(uint32_t thr, bool always)
{
    const uint64_t E = always ? (uint64_t(1) << 32) : (uint64_t)thr;
    const uint64_t A = uint64_t(0) - E;
    return make_uint2((uint32_t)A, (uint32_t)(A >> 32));
}

__device__ __forceinline__ void load_bc_table(BCLds& lds, const BCTable& tbl)
{
    for (uint32_t i = threadIdx.x; i < 256u; i += blockDim.x) {
        const uint32_t key = i >> 4, sj = i & 15u;
        uint2 v = make_uint2(0u, 0u);
        if (key < 6u && sj < 9u) {
            const uint32_t idx = key * 9u + sj;               // ((n * 2 + b) * 9 + sum)
            v = bc_addend(tbl.thr[idx], tbl.always[idx] != 0);
        }
        lds.e[i] = v;
    }
    __syncthreads();
}

// The same from a 96-entry (thr, always) table indexed key * 16 + sum.
__device__ __forceinline__ void load_bc_table(BCLds& lds, const uint2* __restrict__ src96)
{
    for (uint32_t i = threadIdx.x; i < 256u; i += blockDim.x) {
        uint2 v = make_uint2(0u, 0u);
        if (i < 96u) {
            const uint2 e = src96[i];
            if ((i >> 4) < 6u && (i & 15u) < 9u) v = bc_addend(e.x, e.y != 0);
        }
        lds.e[i] = v;
    }
    __syncthreads();
}

template <int HM>
__device__ __forceinline__ uint4 bc_vec(const uint4& src, const uint4& up, const uint4& dn, const uint4& mid,
                                        uint32_t halo, bool odd, uint64_t blk0, uint32_t cb, uint32_t pbits,
                                        uint32_t t, uint32_t color, uint32_t k0, uint32_t k1, uint32_t hu,
                                        const uint2* __restrict__ tab)
{
    uint32_t ev[4], od[4], nxt[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t s = pick(src, d);
        const uint32_t b = spread8(pbits >> (8 * d));
        const uint32_t sum = pick(up, d) + pick(dn, d) + pick(mid, d) + horizontal(mid, d, halo, odd);
        const uint32_t key = s + s + b;                       // n * 2 + b, at most 5 per nibble
        ev[d] = ((key & 0x0F0F0F0Fu) << 4) | (sum & 0x0F0F0F0Fu);     // cells 0, 2, 4, 6 as bytes
        od[d] = (key & 0xF0F0F0F0u) | ((sum >> 4) & 0x0F0F0F0Fu);    // cells 1, 3, 5, 7
        const uint32_t v = s + 0x11111111u + b;               // n + 1 + b in 1..4
        const uint32_t ge3 = ((v + 0x55555555u) & 0x88888888u) >> 3;
        nxt[d] = v - shl_or<1>(ge3, ge3);                     // mod 3
    }
    // nacc = -(accept bits), shifted in cell by cell: 2 (-a) - bit = -(2 a + bit)
    // block indices cb + blk0 + k as in accept_masks
    uint32_t nacc = 0;
    const uint64_t mb = (uint64_t)kPhiloxM0 * cb;
#pragma unroll
    for (int h = 1; h >= 0; --h) {
        Philox4 P[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint64_t b = blk0 + 2 * d + h;
            if (HM == 2)
                P[d] = philox4x32_10(lo32(b), hiw<HM>(b, hu), t, color, k0, k1);
            else
                P[d] = philox4x32_10_p0(mad_m0(lo32(blk0), mb + (uint64_t)kPhiloxM0 * (uint32_t)(2 * d + h)),
                                        hiw<HM>(b, hu), t, color, k0, k1);
        }
#pragma unroll
        for (int jj = 3; jj >= 0; --jj)
#pragma unroll
            for (int d = 3; d >= 0; --d) {
                const int j = 4 * h + jj;
                const uint32_t idx = (((j & 1) ? od[d] : ev[d]) >> (8 * (j >> 1))) & 0xFFu;
                const uint2 e = tab[idx];
                const uint32_t u = philox_word(P[d], jj);
                nacc = shl_add<1>(nacc, add_hi(u, ((uint64_t)e.y << 32) | e.x));
            }
    }
    const uint32_t acc = 0u - nacc;
    uint32_t res[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t s = pick(src, d);
        const uint32_t a = (acc >> d) & 0x11111111u;
        const uint32_t mask = shl_opaque<4>(a) - a;           // 0xF in accepted nibbles
        res[d] = (s & ~mask) | (nxt[d] & mask);
    }
    return make_uint4(res[0], res[1], res[2], res[3]);
}

// ---------------------------------------------------------------------------
// Half-sweep: one thread per 16-byte column vector, walking `rows` rows
// (even, starting at an even row).  The colour is a template parameter, so
// the parity of y + c, which picks the horizontal neighbours, is known at
// compile time for the two rows of each unrolled pair.
// ---------------------------------------------------------------------------
struct RowState {
    const uint4* pcur;      // other plane, row y, this column
    uint4* pown;            // own plane, row y, this column
    const uint32_t* hrow;   // other plane, row y, word 0
    uint64_t blk;           // accept block of the vector's cell 0
    uint64_t kv;            // in-colour index of the vector's cell 0
    uint4 up, mid;
};

template <int MODEL, int HM, bool ODD>
__device__ __forceinline__ void row_step(RowState& st, const uint4* __restrict__ oth_col0, uint32_t y, uint32_t L,
                                         uint32_t Q, uint32_t W, uint32_t hwl, uint32_t hwr, uint32_t color,
                                         uint32_t t, uint32_t k0, uint32_t k1, uint32_t hu, uint32_t T4, uint32_t T8,
                                         const uint2* tab)
{
    const uint4* pdn = (y + 1 == L) ? oth_col0 : st.pcur + Q;
    const uint4 dn = *pdn;
    const uint4 src = *st.pown;
    const uint32_t halo = st.hrow[ODD ? hwr : hwl];
    uint4 res;
    if (MODEL == 0) {
        res = ising_vec<HM>(src, st.up, dn, st.mid, halo, ODD, st.blk, 0u, t, color, k0, k1, hu, T4, T8);
    } else {
        const uint64_t pb = st.kv >> 7;
        const Philox4 p = philox4x32_10(lo32(pb), HM == 0 ? 0u : hi32(pb), t, 2u + color, k0, k1);
        const uint32_t pbits = philox_word(p, (int)((st.kv >> 5) & 3));
        res = bc_vec<HM>(src, st.up, dn, st.mid, halo, ODD, st.blk, 0u, pbits, t, color, k0, k1, hu, tab);
    }
    *st.pown = res;
    st.up = st.mid;
    st.mid = dn;
    st.pcur += Q;
    st.pown += Q;
    st.hrow += W;
    st.blk += L >> 3;
    st.kv += L >> 1;
}

// One thread's share of a half-sweep: column vector q of rows
// [y0, y0 + rows) of an L x L lattice (rows even, y0 even).
template <int MODEL, int HM, int COLOR>
__device__ __forceinline__ void band_update(uint32_t* __restrict__ own, const uint32_t* __restrict__ oth, uint32_t L,
                                            uint32_t rows, uint32_t q, uint32_t y0, uint32_t t, uint32_t k0,
                                            uint32_t k1, uint32_t hu, uint32_t T4, uint32_t T8, const uint2* tab)
{
    const uint32_t Q = L >> 6;
    const uint32_t W = L >> 4;
    const uint4* __restrict__ oth4 = reinterpret_cast<const uint4*>(oth) + q;
    RowState st;
    st.pcur = oth4 + (size_t)y0 * Q;
    st.pown = reinterpret_cast<uint4*>(own) + (size_t)y0 * Q + q;
    st.hrow = oth + (size_t)y0 * W;
    st.blk = ((uint64_t)y0 * (L >> 1) + 32u * q) >> 2;
    st.kv = (uint64_t)y0 * (L >> 1) + 32u * q;
    st.up = *(oth4 + (size_t)(y0 == 0 ? L - 1 : y0 - 1) * Q);
    st.mid = *st.pcur;
    const uint32_t hwl = (q == 0) ? W - 1 : 4 * q - 1;         // word left of the vector
    const uint32_t hwr = (4 * q + 4 == W) ? 0 : 4 * q + 4;     // word right of the vector
    for (uint32_t r = 0; r < rows; r += 2) {
        // even row y: parity of y + c is c; odd row: 1 - c
        row_step<MODEL, HM, COLOR == 1>(st, oth4, y0 + r, L, Q, W, hwl, hwr, COLOR, t, k0, k1, hu, T4, T8, tab);
        row_step<MODEL, HM, COLOR == 0>(st, oth4, y0 + r + 1, L, Q, W, hwl, hwr, COLOR, t, k0, k1, hu, T4, T8, tab);
    }
}

// ---------------------------------------------------------------------------
// The same walk for a wave whose 64 lanes hold 64 consecutive column vectors
// of one band (L a multiple of 4096, so a row holds a whole number of waves):
// the row, its addresses, the periodic wrap in y and the Philox counters'
// row terms are wave-uniform and stay in scalar registers, and a lane keeps
// only its byte offsets in a row and its counter offsets from the wave's
// first block.  The wave's accept blocks of a row are the 512 indices from
// y L/8 + 8 q0 (q0 = q rounded down to 64, a multiple of 512 since L/8 is),
// so cb + 8 (q - q0) + k never carries into the high word, which is one
// value per wave and row; its proposal blocks (Blume-Capel) are the 16
// indices from y L/256 + q0/4, likewise aligned.
// ---------------------------------------------------------------------------
struct WaveLane {
    uint32_t qo;        // byte offset of the lane's vector in a row
    uint32_t hl, hr;    // byte offsets of the words left and right of it
    uint32_t a8;        // 8 (q - q0): accept-block offset in the wave's row
    uint32_t p4;        // (q - q0) / 4: proposal-block offset
    uint32_t sel;       // q & 3: the proposal block's output word
};

__device__ __forceinline__ uint4 load_row(const char* row, uint32_t off)
{
    return *reinterpret_cast<const uint4*>(row + off);
}

template <int MODEL, bool HI0, bool ODD>
__device__ __forceinline__ void row_step_wave(const WaveLane& w, const char* oth, char* own, uint32_t y, uint32_t L,
                                              uint32_t q0, uint4& up, uint4& mid, uint32_t color, uint32_t t,
                                              uint32_t k0, uint32_t k1, uint32_t T4, uint32_t T8, const uint2* tab)
{
    const uint64_t rowb = L >> 2;                       // bytes per row of a plane
    // keep the lane offsets' widening next to each access, where it forms
    // the scalar-base + 32-bit-offset address of global loads and stores
    uint32_t qo = w.qo, ho = ODD ? w.hr : w.hl;
    asm volatile("" : "+v"(qo), "+v"(ho));
    const char* orow = oth + (uint64_t)y * rowb;
    const char* odn = (y + 1 == L) ? oth : orow + rowb;
    char* wrow = own + (uint64_t)y * rowb;
    const uint4 dn = load_row(odn, qo);
    const uint4 src = load_row(wrow, qo);
    const uint32_t halo = *reinterpret_cast<const uint32_t*>(orow + ho);
    const uint64_t bw = (uint64_t)y * (L >> 3) + 8u * q0;
    constexpr int HM = HI0 ? 0 : 1;
    uint4 res;
    if (MODEL == 0) {
        res = ising_vec<HM>(src, up, dn, mid, halo, ODD, w.a8, lo32(bw), t, color, k0, k1, hi32(bw), T4, T8);
    } else {
        const uint64_t pw = (uint64_t)y * (L >> 8) + (q0 >> 2);
        const Philox4 p = philox4x32_10_p0(mad_m0(w.p4, (uint64_t)kPhiloxM0 * lo32(pw)), HI0 ? 0u : hi32(pw), t,
                                           2u + color, k0, k1);
        const uint32_t pbits = philox_word(p, (int)w.sel);
        res = bc_vec<HM>(src, up, dn, mid, halo, ODD, w.a8, lo32(bw), pbits, t, color, k0, k1, hi32(bw), tab);
    }
    *reinterpret_cast<uint4*>(wrow + qo) = res;
    up = mid;
    mid = dn;
}

template <int MODEL, bool HI0, int COLOR>
__device__ __forceinline__ void band_update_wave(uint32_t* __restrict__ own, const uint32_t* __restrict__ oth,
                                                 uint32_t L, uint32_t rows, uint32_t q, uint32_t y0, uint32_t t,
                                                 uint32_t k0, uint32_t k1, uint32_t T4, uint32_t T8, const uint2* tab)
{
    const uint32_t W = L >> 4;
    const uint32_t q0 = __builtin_amdgcn_readfirstlane(q & ~63u);
    y0 = __builtin_amdgcn_readfirstlane(y0);
    WaveLane w;
    w.qo = q << 4;
    w.hl = ((q == 0) ? W - 1 : 4 * q - 1) << 2;
    w.hr = ((4 * q + 4 == W) ? 0 : 4 * q + 4) << 2;
    w.a8 = (q & 63u) << 3;
    w.p4 = (q & 63u) >> 2;
    w.sel = q & 3u;
    const char* ob = reinterpret_cast<const char*>(oth);
    char* wb = reinterpret_cast<char*>(own);
    const uint64_t rowb = L >> 2;
    uint4 up = load_row(ob + (uint64_t)(y0 == 0 ? L - 1 : y0 - 1) * rowb, w.qo);
    uint4 mid = load_row(ob + (uint64_t)y0 * rowb, w.qo);
    for (uint32_t r = 0; r < rows; r += 2) {
        row_step_wave<MODEL, HI0, COLOR == 1>(w, ob, wb, y0 + r, L, q0, up, mid, COLOR, t, k0, k1, T4, T8, tab);
        row_step_wave<MODEL, HI0, COLOR == 0>(w, ob, wb, y0 + r + 1, L, q0, up, mid, COLOR, t, k0, k1, T4, T8, tab);
    }
}

// ---------------------------------------------------------------------------
// 1-bit Ising with table-driven random bits (section 3.2).  Cells are single
// bits (1 for s = +1), 32 per word, 128 per 16-byte vector.  For a word of
// 32 cells:
//   b_n = neighbour word ^ own word marks the misaligned neighbours; with
//   half adders over the four b_n, eq4 = no mismatch and eq3 = exactly one;
//   exp4 = the 4-bit patterns of 8 table draws (stream 0), exp8 = those of
//   stream 1 ANDed with exp4 (probability e^{-8 beta}); a cell keeps its
//   value iff eq4 with no exp8 bit or eq3 with no exp4 bit, all others flip.
// Table search: T is the 16-entry table clamped to 2^32 - 1 (in LDS), kmax
// the last entry that was below 2^32; the pattern is min(k, kmax) with k
// the largest index whose clamped entry is <= u, which equals the largest
// index whose exact entry is <= u.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lut_lookup(const uint32_t* __restrict__ T, uint32_t T8, uint32_t kmax, uint32_t u)
{
    uint32_t k = (u >= T8) ? 8u : 0u;
    k += (u >= T[k + 4]) ? 4u : 0u;
    k += (u >= T[k + 2]) ? 2u : 0u;
    k += (u >= T[k + 1]) ? 1u : 0u;
    return k < kmax ? k : kmax;
}

// Random bits of 32 cells (8 groups of 4) from the 8 draws of two Philox
// blocks P, R, by the exact table search.
__device__ __forceinline__ uint32_t lut_word(const Philox4& P, const Philox4& R, const uint32_t* __restrict__ T,
                                             uint32_t T8, uint32_t kmax)
{
    uint32_t w = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        w |= lut_lookup(T, T8, kmax, philox_word(j < 4 ? P : R, j & 3)) << (4 * j);
    return w;
}

// Bucketed lookup.  Bucket b = u >> 20 (4096 buckets) holds a 64-bit
// addend A = kw 2^32 + 2^32 - Tn with max{k : T[k] <= u} = kw + [u >= Tn] =
// the high word of u + A for every u of the bucket.  Buckets where no such
// pair exists (two or more thresholds inside) hold A = 2^63, and a word
// with any such draw takes the exact search instead.
constexpr int kLutBuckets = 4096;

// Entry of bucket b: for the draws u of [lo, hi] = [b 2^20, b 2^20 + 2^20 - 1],
// klo = max{k <= kmax : T[k] <= lo} and `inner` counts the thresholds in
// (lo, hi].  The sorted table makes the answer klo below the one inner
// threshold T[klo + 1] and klo + 1 from it on; with none inside it is klo
// throughout.
__device__ __forceinline__ uint64_t lut_bucket_addend(const uint32_t* T, uint32_t kmax, uint32_t b)
{
    const uint32_t lo = b << 20, hi = lo + 0xFFFFFu;
    uint32_t klo = 0, inner = 0;
    for (uint32_t k = 1; k < 16; ++k) {
        if (k > kmax) break;
        if (T[k] <= lo) klo = k;
        else if (T[k] <= hi) ++inner;
    }
    // the answer is kw + [u >= Tn] on the bucket; stored as kw 2^32 + 2^32 - Tn
    if (inner == 1 || (inner == 0 && klo < kmax))
        return ((uint64_t)klo << 32) + (uint64_t(1) << 32) - T[klo + 1];    // next threshold
    if (inner == 0 && hi != 0xFFFFFFFFu) return ((uint64_t)klo << 32) + 1u;   // Tn = 2^32 - 1, above the bucket
    if (inner == 0 && klo >= 1) return (uint64_t)klo << 32;                     // kw = klo - 1, Tn = 0
    return uint64_t(1) << 63;                                                   // exact search
}

// Pattern of draw i (0..7) of a word: bits 4i .. 4i + 3, placed with one
// v_lshl_or_b32 (a pattern is at most 15 on the fast path; a marked bucket
// sets bit 31 of k, which `flags` collects).
template <int I>
__device__ __forceinline__ void lut_fast_draw(uint32_t u, const uint2* __restrict__ B, uint32_t& w, uint32_t& flags)
{
    const uint2 e = B[u >> 20];
    const uint32_t k = add_hi(u, ((uint64_t)e.y << 32) | e.x);
    flags |= k;
    w = shl_or<4 * I>(k, w);
}

// Random bits of the 32 cells whose 8 groups of 4 start at group g0 (a
// multiple of 8): Philox blocks g0/4 and g0/4 + 1 of `stream`.
template <int HM>
__device__ __forceinline__ uint32_t lut_word_fast(uint64_t g0, uint32_t t, uint32_t stream, uint32_t k0, uint32_t k1,
                                                  uint32_t hu, const uint2* __restrict__ B,
                                                  const uint32_t* __restrict__ T, uint32_t T8, uint32_t kmax)
{
    uint32_t w = 0, flags = 0;
    const uint64_t b = g0 >> 2;
    const Philox4 P = philox4x32_10(lo32(b), hiw<HM>(b, hu), t, stream, k0, k1);
    const Philox4 R = philox4x32_10(lo32(b + 1), hiw<HM>(b + 1, hu), t, stream, k0, k1);
    lut_fast_draw<0>(P.v0, B, w, flags);
    lut_fast_draw<1>(P.v1, B, w, flags);
    lut_fast_draw<2>(P.v2, B, w, flags);
    lut_fast_draw<3>(P.v3, B, w, flags);
    lut_fast_draw<4>(R.v0, B, w, flags);
    lut_fast_draw<5>(R.v1, B, w, flags);
    lut_fast_draw<6>(R.v2, B, w, flags);
    lut_fast_draw<7>(R.v3, B, w, flags);
    if (flags >> 31) w = lut_word(P, R, T, T8, kmax);
    return w;
}

template <int HM>
__device__ __forceinline__ uint4 lut_vec(const uint4& src, const uint4& up, const uint4& dn, const uint4& mid,
                                         uint32_t halo, bool odd, uint64_t kv, uint32_t t, uint32_t color,
                                         uint32_t k0, uint32_t k1, uint32_t hu, const uint2* __restrict__ B,
                                         const uint32_t* __restrict__ T, uint32_t T8, uint32_t kmax)
{
    uint32_t res[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t s = pick(src, d);
        const uint32_t w = pick(mid, d);
        const uint32_t hs = odd ? funnel(d < 3 ? pick(mid, d + 1) : halo, w, 1)
                                : funnel(w, d > 0 ? pick(mid, d - 1) : halo, 31);
        const uint32_t b0 = pick(up, d) ^ s, b1 = pick(dn, d) ^ s, b2 = w ^ s, b3 = hs ^ s;
        const uint32_t t1 = b0 ^ b1, u1 = b0 & b1, t2 = b2 ^ b3, u2 = b2 & b3;
        const uint32_t eq4 = ~(b0 | b1 | b2 | b3);
        const uint32_t eq3 = (t1 ^ t2) & ~(u1 | u2);
        const uint64_t g0 = (kv + 32u * d) >> 2;
        const uint32_t e4 = lut_word_fast<HM>(g0, t, 8u + 2u * color, k0, k1, hu, B, T, T8, kmax);
        const uint32_t e8 = lut_word_fast<HM>(g0, t, 9u + 2u * color, k0, k1, hu, B, T, T8, kmax) & e4;
        // a spin keeps its value only when four neighbours agree and its
        // e^{-8 beta} bit is clear, or three agree and its e^{-4 beta} bit is clear
        const uint32_t keep = (eq4 & ~e8) | (eq3 & ~e4);
        res[d] = ~(s ^ keep);
    }
    return make_uint4(res[0], res[1], res[2], res[3]);
}

// One thread's share of a 1-bit half-sweep: column vector q (128 cells) of
// rows [y0, y0 + rows) (rows even, y0 even).
template <int HM, int COLOR>
__device__ __forceinline__ void band_update_lut(uint32_t* __restrict__ own, const uint32_t* __restrict__ oth,
                                                uint32_t L, uint32_t rows, uint32_t q, uint32_t y0, uint32_t t,
                                                uint32_t k0, uint32_t k1, uint32_t hu, const uint2* B,
                                                const uint32_t* T, uint32_t T8, uint32_t kmax)
{
    const uint32_t Q = L >> 8;                  // 16-byte vectors per row
    const uint32_t W = L >> 6;                  // words per row
    const uint4* __restrict__ oth4 = reinterpret_cast<const uint4*>(oth) + q;
    const uint4* pcur = oth4 + (size_t)y0 * Q;
    uint4* pown = reinterpret_cast<uint4*>(own) + (size_t)y0 * Q + q;
    const uint32_t* hrow = oth + (size_t)y0 * W;
    uint64_t kv = (uint64_t)y0 * (L >> 1) + 128u * q;
    uint4 up = *(oth4 + (size_t)(y0 == 0 ? L - 1 : y0 - 1) * Q);
    uint4 mid = *pcur;
    const uint32_t hwl = (q == 0) ? W - 1 : 4 * q - 1;
    const uint32_t hwr = (4 * q + 4 == W) ? 0 : 4 * q + 4;
    for (uint32_t r = 0; r < rows; ++r) {
        const uint32_t y = y0 + r;
        const bool odd = ((y + COLOR) & 1u) != 0;
        const uint4 dn = *((y + 1 == L) ? oth4 : pcur + Q);
        const uint4 src = *pown;
        const uint32_t halo = hrow[odd ? hwr : hwl];
        *pown = lut_vec<HM>(src, up, dn, mid, halo, odd, kv, t, COLOR, k0, k1, hu, B, T, T8, kmax);
        up = mid;
        mid = dn;
        pcur += Q;
        pown += Q;
        hrow += W;
        kv += L >> 1;
    }
}

// The counter mode of a thread's band whose Philox blocks run from b_first
// to b_last: 0 while every block index of the lattice fits 32 bits (hi0),
// else 1 with hu the high word when the whole wave shares it (for L a
// power of two it changes only between bands), else 2 (per lane).
__device__ __forceinline__ int counter_mode(bool hi0, uint64_t b_first, uint64_t b_last, uint32_t& hu)
{
    hu = 0;
    if (hi0) return 0;
    const uint32_t hf = hi32(b_first);
    hu = __builtin_amdgcn_readfirstlane(hf);
    return __all(hf == hu && hi32(b_last) == hu) ? 1 : 2;
}

}  // namespace dev
}  // namespace mcl
