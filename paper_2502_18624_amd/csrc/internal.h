// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mcl {

// Geometry of one lattice in device memory (layout described in common.h).
struct Geom {
    int64_t L;          // linear size, multiple of 64 (256 for 1-bit cells)
    int64_t W;          // 32-bit words per plane row: L / 16 (4-bit cells), L / 64 (1-bit)
    int64_t Q;          // 16-byte vectors per plane row: L / 64 (4-bit cells), L / 256 (1-bit)
    int cb;             // bits per cell: 4 or 1
    uint32_t* plane0;   // colour 0 cells; colour 1 follows at plane0 + L * W
    uint32_t* plane(int c) const { return plane0 + (c ? L * W : 0); }
    int64_t plane_words() const { return L * W; }
};

// Write the initial state into both planes.
hipError_t launch_init(const Geom& g, int model, int init_state, uint64_t seed, hipStream_t s);

// One colour of one sweep.
struct HalfSweepArgs {
    int color;
    uint32_t t;             // sweep index, or its offset from *tbase when tbase is set
    const uint32_t* tbase;  // device word added to t by the kernel (nullptr: t is absolute)
    uint64_t seed;
    uint32_t T4, T8;        // Ising thresholds (e^{-4 beta}, e^{-8 beta})
    const BCTable* bc;      // Blume-Capel table (host copy, passed by value)
};
hipError_t launch_ising_half(const Geom& g, const HalfSweepArgs& a, hipStream_t s);
// 1-bit Ising with table-driven random bits (W = L/64, Q = L/256 in Geom).
hipError_t launch_init1(const Geom& g, int init_state, uint64_t seed, hipStream_t s);
// Bucket table of the 1-bit mode: kLutBucketBytes of device memory, built
// once per beta, read by every half-sweep at that beta.
constexpr int64_t kLutBucketBytes = 4096 * 8;
hipError_t launch_lut_buckets(const LutTable& tab, void* buckets, hipStream_t s);
hipError_t launch_lut_half(const Geom& g, int color, uint32_t t, const uint32_t* tbase, uint64_t seed,
                           const LutTable& tab, const void* buckets, hipStream_t s);
hipError_t launch_bc_half(const Geom& g, const HalfSweepArgs& a, hipStream_t s);
// One device word: *p = v, or *p += v with add (a one-lane kernel, so that
// it can sit in a captured graph).
hipError_t launch_set_word(uint32_t* p, uint32_t v, bool add, hipStream_t s);

// Measurement kernels accumulating into int64 device scratch.
// acc layout: [0] B, [1] M (from +1 count minus -1 count), [2] #(+1),
// [3] #(-1), [4] #(0), [5..15] reserved; cells that are none of the three
// (corrupted) are L^2 minus the three counts.
constexpr int kAccSlots = 16;
hipError_t launch_zero(int64_t* p, int64_t n, hipStream_t s);
// T bits of the sampled columns x = 0 mod 16: for every row y, bit j of
// word k is [s(16 (32 k + j), y) = +1] (and, Blume-Capel only, a second
// plane of [s != 0] after L rows); tbits_words(L) words per row, the L / 16
// bits of a row repeated to fill one word below L = 512 (L is a power of
// two wherever they are used; other L get room for ceil(L / 512) words).
// 4-bit Ising lattices have room after the L rows for the residue rows of
// the sampled rows: row 16 b + rho holds, for y = 16 b, bit j of word k =
// [s(16 (32 k + j) + rho, y) = +1] (written by the fused short-distance
// tiles, read by the sampled x pass).
inline int64_t tbits_words(int64_t L) { return L >= 512 ? (L + 511) / 512 : 1; }
inline int64_t tbits_bytes(int model, int64_t L) { return (model == 2 ? 1 : 2) * L * tbits_words(L) * 4; }
// B, M, Q, counts and the sigma-h histogram into acc; with tbits set, also
// the T bits of every row (written by the same pass from L = 512 on).
hipError_t launch_bmq(const Geom& g, int model, int64_t* acc, uint32_t* tbits, hipStream_t s);
// Correlations from every source at r = 0..R (R <= 32), LDS-tiled.  With acc
// set (4-bit Ising cells, L >= 4096, see bmq_fused) the same tiles give what
// launch_bmq adds to acc, and with tbits set (L a power of two) the T bits
// and the residue rows of the sampled rows after them;
// acc[14] then counts the workgroups that met a cell holding no spin, for
// which the caller must run launch_bmq instead (acc zeroed, tbits null).
hipError_t launch_corr_short(const Geom& g, int model, int R, int64_t* Cx, int64_t* Cy, int64_t* acc,
                             uint32_t* tbits, hipStream_t s);
// Whether measure() takes B/M/Q from the short-distance tiles when it runs
// them: 4-bit Ising cells at L >= 4096, unless the environment variable
// MCL_MEASURE_FUSED is 0 (read at every call).  For 1-bit cells the B/M/Q
// pass reads a quarter of the bytes and stays the cheaper way.
bool bmq_fused(const Geom& g, int model);
// Correlations from every source at distances r[0..nr) (any r <= L/2).
hipError_t launch_corr_all(const Geom& g, const int32_t* r_dev, int nr, int64_t* Cx, int64_t* Cy,
                           hipStream_t s);
// Correlations from the sampled sources x = y = 0 (mod 16) at r[0..nr), from
// the lattice (x) and the T bits of the B/M/Q pass (y).
struct SampledArgs {
    const int32_t* r;
    int nr;
    int64_t* Cx;
    int64_t* Cy;
    const uint32_t* tbits;
    const uint32_t* rbits = nullptr;    // residue rows (4-bit Ising, written by the fused tiles), or null
    int nlin = 0;                       // r[0 .. nlin) = rlin0, rlin0 + 1, ... (consecutive distances)
    uint32_t rlin0 = 0;
};
// The sampled sources' two passes: x (the lattice's sampled rows, or the
// residue rows when rbits is set) and y (the T bits only).  They are
// independent, so the caller may run them on two streams.
hipError_t launch_corr_sampled_x(const Geom& g, int model, const SampledArgs& a, hipStream_t s);
hipError_t launch_corr_sampled_y(const Geom& g, int model, const SampledArgs& a, hipStream_t s);

// Batched half-sweep.  One descriptor per replica (64 bytes).  The work of
// a launch is a list of tiles of 256 threads; replica i owns the tiles
// [tile_begin, next replica's tile_begin).  A thread of a tile is one
// 16-byte column vector (32 four-bit or 128 one-bit cells) of one band of
// `rows` rows, as in the one-lattice kernels.
struct GroupDesc {
    uint32_t* plane0;      // the replica's planes (P_1 follows P_0)
    uint32_t L;
    uint32_t rows;         // band rows: even, divides L
    uint32_t t0;           // sweep counter at the start of the call
    uint32_t n;            // sweeps for this replica in this call
    uint32_t k0, k1;       // Philox key (seed)
    uint32_t T4, T8;       // Ising thresholds (4-bit Ising)
    uint32_t tile_begin;   // first tile of this replica in its launch
    uint32_t model;        // 0: Ising 4-bit, 1: Blume-Capel, 2: Ising 1-bit
    uint32_t tab;          // Blume-Capel: index of its 96-entry table; 1-bit: index of its LutRec
    uint32_t pad[3];
};
static_assert(sizeof(GroupDesc) == 64, "descriptor size");

// Table of a 1-bit replica in the batched path: its bucket table (in the
// replica's own device buffer, rebuilt per call) and the 16 clamped
// thresholds with the last index below 2^32.
struct LutRec {
    uint2* buckets;
    uint32_t T[16];
    uint32_t kmax;
    uint32_t pad;
};
static_assert(sizeof(LutRec) == 80, "1-bit record size");

// Models a batched launch may hold (bit m for model m).  A launch whose mask
// has one bit runs that model's path only (and its register budget).
constexpr int kMaskIsing = 1, kMaskBC = 2, kMaskLut = 4;

// One colour of sweep s (+ *sbase when sbase is set) for every replica of
// the list with s < n; grid workgroups (a multiple of 8) walk the `total`
// tiles, each XCD's workgroups one contiguous eighth of the list.  With
// fewer workgroups than tiles they claim tiles from the 16 counter words at
// ctr, which must be zero before the first such launch and are zero again
// after each (nullptr: a fixed share per workgroup).
hipError_t launch_group_half(int mask, int color, const GroupDesc* desc, int count, uint32_t total,
                             uint32_t grid, const uint2* bc_tables, const LutRec* luts, uint32_t s,
                             const uint32_t* sbase, uint32_t* ctr, hipStream_t st);
// Bucket tables of the 1-bit replicas of a batched call.
hipError_t launch_group_lut_buckets(const LutRec* luts, int n, hipStream_t st);

}  // namespace mcl
