// Device-side building blocks shared by the library's kernels (gfx950).
//
// Storage layout of one lattice (L a multiple of 64):
//   two colour planes P_0, P_1 (checkerboard decomposition, section 3.1);
//   plane c holds the sites of colour c = (x + y) & 1, row-major, L rows of
//   L/2 cells, the cell of site (x, y) at in-plane index i = x >> 1;
//   4 bits per cell, 8 cells per 32-bit word (cell i in bits 4(i&7)..+3 of
//   word i >> 3), so a row is L/16 words = L/64 16-byte vectors;
//   cell value n = s + 1 (Ising uses 0 and 2, Blume-Capel 0, 1, 2), so the
//   sum of four neighbour cells is at most 8 and fits its nibble (the
//   multi-spin coding of section 3.2).
//   Plane P_1 follows P_0 directly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcl {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// a ^ b ^ c in one VALU instruction (v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// products and xors, key advanced by the Weyl constants between rounds.
// Each product is one v_mad_u64_u32 and each pair of xors one v_bitop3_b32.
// The first two rounds use plain xors: when the caller's counter words 1..3
// and key are wave-uniform (the sweep index, the stream and a zero high
// word), the compiler moves half of those rounds' work to the scalar unit.
struct Philox4 {
    uint32_t v0, v1, v2, v3;
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        uint32_t n0, n2;
        if (r < 2) {
            n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        } else {
            n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
            n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        }
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return Philox4{c0, c1, c2, c3};
}

// The same with the first round's product M0 * c0 given (a caller whose
// counters differ by a constant k can pass M0 * c + M0 * k, one multiply-add
// with a constant addend, instead of adding k to the counter first).
__device__ __forceinline__ Philox4 philox4x32_10_p0(uint64_t p0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                    uint32_t k1)
{
    uint32_t c0;
    {
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        const uint64_t q0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t q1 = (uint64_t)kPhiloxM1 * c2;
        uint32_t n0, n2;
        if (r < 2) {
            n0 = (uint32_t)(q1 >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(q0 >> 32) ^ c3 ^ k1;
        } else {
            n0 = xor3((uint32_t)(q1 >> 32), c1, k0);
            n2 = xor3((uint32_t)(q0 >> 32), c3, k1);
        }
        c1 = (uint32_t)q1;
        c3 = (uint32_t)q0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return Philox4{c0, c1, c2, c3};
}

// M0 * c + a (64-bit) in one v_mad_u64_u32, with the constant addend a in
// scalar registers and M0 in a vector register (a VOP3 reads one scalar
// operand; left to itself the compiler keeps M0 scalar and copies each
// addend into vector registers on every use).
__device__ __forceinline__ uint64_t mad_m0(uint32_t c, uint64_t a)
{
    uint64_t d;
    asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(d) : "v"(c), "v"(kPhiloxM0), "s"(a) : "vcc");
    return d;
}

// (a ^ b) + c in one VALU instruction (v_xad_u32).  Written out, a chain of
// these is re-associated into separate xors and three-input adds.
__device__ __forceinline__ uint32_t xad(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_xad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t philox_word(const Philox4& p, int i)
{
    return i == 0 ? p.v0 : i == 1 ? p.v1 : i == 2 ? p.v2 : p.v3;
}

// acc * 2 + [u < T]: the comparison's carry goes straight into an
// add-with-carry (two VALU instructions; T must live in an SGPR).  Left to
// itself the compiler builds such masks with compare, select and or.
__device__ __forceinline__ uint32_t shift_in_lt(uint32_t acc, uint32_t u, uint32_t T)
{
    uint32_t r;
    asm("v_cmp_gt_u32_e32 vcc, %2, %1\n\t"
        "v_addc_co_u32_e32 %0, vcc, %3, %3, vcc"
        : "=v"(r)
        : "v"(u), "s"(T), "v"(acc)
        : "vcc");
    return r;
}

// High word of u + A (64-bit; one v_mad_u64_u32 with multiplier 1).  With
// A = -E for E in [0, 2^32] it is -[u < E]: a 33-bit comparison in one
// instruction.
__device__ __forceinline__ uint32_t add_hi(uint32_t u, uint64_t A)
{
    uint64_t d;
    asm("v_mad_u64_u32 %0, vcc, %1, 1, %2" : "=v"(d) : "v"(u), "v"(A) : "vcc");
    return (uint32_t)(d >> 32);
}

// (x << S) | y as one v_lshl_or_b32.  Written out, an or of disjoint
// shifted copies (or x << 4 minus x) is turned by the compiler into a
// quarter-rate v_mul_lo_u32 by a constant.
template <int S>
__device__ __forceinline__ uint32_t shl_or(uint32_t x, uint32_t y)
{
    uint32_t r;
    asm("v_lshl_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "i"(S), "v"(y));
    return r;
}

// (x << S) + y as one v_lshl_add_u32 (a chain of these is otherwise
// re-associated into multiplies).
template <int S>
__device__ __forceinline__ uint32_t shl_add(uint32_t x, uint32_t y)
{
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "i"(S), "v"(y));
    return r;
}

template <int S>
__device__ __forceinline__ uint32_t shl_opaque(uint32_t x)
{
    return shl_or<S>(x, 0u);
}

// ({hi, lo} >> sh)[31:0], sh in 0..31 (one v_alignbit_b32).
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// Number of set bits.
__device__ __forceinline__ uint32_t popc(uint32_t v) { return __builtin_popcount(v); }

// Sum over the 8 cell pairs of two words of s * s', s = n - 1 for n in
// {0, 1, 2}: a product is nonzero iff neither cell is 1 (bit 0 clear in
// both) and is +1 iff their bit 1 agrees.
__device__ __forceinline__ int pair_products(uint32_t a, uint32_t b)
{
    const uint32_t nz = ~(a | b) & 0x11111111u;
    const uint32_t diff = ((a ^ b) >> 1) & nz;
    return (int)popc(nz) - 2 * (int)popc(diff);
}

__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the active lanes of the wave, returned to every lane (the device
// library's wavefront reduction: DPP row operations, no LDS permutes).
__device__ __forceinline__ int wave_sum_i32(int v) { return __ockl_wfred_add_i32(v); }

// Blume-Capel acceptance table entry: threshold and "always accept" flag
// (dE <= 0), indexed ((n * 2) + b) * 9 + neighbour-cell-sum, n = s + 1.
struct BCTable {
    uint32_t thr[54];
    uint32_t always[54];
};

// Table of the 1-bit Ising mode: the 16 sorted thresholds clamped to
// 2^32 - 1 and the last index whose exact value was below 2^32.
struct LutTable {
    uint32_t T[16];
    uint32_t kmax;
};

}  // namespace mcl
