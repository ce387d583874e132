// Batched half-sweep: many independent lattices -- any mix of models,
// sizes, temperatures, crystal fields and seeds -- advance in one launch per
// colour.  The work is a list of tiles of 256 threads; every tile belongs to
// one replica, so the replica's parameters are wave-uniform, and the
// per-thread work is the one-lattice band update of sweep_device.h: every
// lattice ends bit-identical to its own sweeps.
//
// The grid is one workgroup per tile or persistent: `grid` workgroups (a
// multiple of 8) walking the tile list.  Workgroup ids go round-robin to
// the 8 XCDs, so the workgroups of XCD x take the tiles of the x-th eighth
// of the list; neighbouring tiles of a replica (whose bands share halo rows)
// then run on one XCD and meet in its L2.  A persistent grid claims the
// tiles of its eighth one at a time from a counter (tiles differ in cost by
// model and band height, so a fixed share per workgroup leaves some of them
// late); the last workgroup of an eighth to find it empty resets the
// counters for the next launch.  A workgroup keeps the acceptance table of
// its current replica in LDS and reloads it only when its next tile belongs
// to another replica: the 96-entry Blume-Capel table, or the 32 KiB bucket
// table of a 1-bit replica.
#include "internal.h"
#include "sweep_device.h"

namespace mcl {
namespace {

// Replica of tile `tile`: last descriptor with tile_begin <= tile.
__device__ __forceinline__ int find_replica(const GroupDesc* __restrict__ desc, int count, uint32_t tile)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].tile_begin <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct LutLds {
    uint2 b[dev::kLutBuckets];
    uint32_t T[16];
};

// LDS of a launch: the Blume-Capel table, or (launches holding 1-bit
// replicas) room for either table.
template <bool LUT>
union GroupLds;

template <>
union GroupLds<false> {
    dev::BCLds bc;
};

template <>
union GroupLds<true> {
    dev::BCLds bc;
    LutLds lut;
};

template <int MASK>
__device__ __forceinline__ uint32_t model_of(uint32_t m)
{
    return MASK == kMaskIsing ? 0u : MASK == kMaskBC ? 1u : MASK == kMaskLut ? 2u : m;
}

// At most 128 VGPRs (4 waves per SIMD): the launches that hold Ising and
// Blume-Capel replicas together would otherwise take 131 and run 3 waves;
// the few values this spills are kept across a tile, not inside its rows.
// ctr: 16 words, zero before the launch (claim counters of the eighths,
// then their counts of workgroups done), for a persistent grid; nullptr for
// a fixed walk.
template <int MASK, int COLOR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void group_half_kernel(
    const GroupDesc* __restrict__ desc, int count, const uint2* __restrict__ bc_tables,
    const LutRec* __restrict__ luts, uint32_t total, uint32_t s, const uint32_t* __restrict__ sbase,
    uint32_t* __restrict__ ctr)
{
    constexpr bool kLut = (MASK & kMaskLut) != 0;
    __shared__ GroupLds<kLut> lds;
    __shared__ uint32_t s_claim;
    if (sbase) s += *sbase;
    // a grid that is not a multiple of 8 walks the whole list round-robin
    const bool by_xcd = (gridDim.x & 7u) == 0;
    const uint32_t part = by_xcd ? (blockIdx.x & 7u) : 0u;
    const uint32_t slot = by_xcd ? (blockIdx.x >> 3) : blockIdx.x;
    const uint32_t step = by_xcd ? (gridDim.x >> 3) : gridDim.x;
    const uint32_t seg_begin = by_xcd ? (uint32_t)((uint64_t)total * part / 8u) : 0u;
    const uint32_t seg_len = (by_xcd ? (uint32_t)((uint64_t)total * (part + 1u) / 8u) : total) - seg_begin;
    const bool claim = ctr != nullptr && by_xcd;
    int cur = -1;                                   // replica whose table is in LDS
    for (uint32_t next = slot;;) {
        uint32_t k;
        if (claim) {
            if (threadIdx.x == 0) s_claim = atomicAdd(&ctr[part], 1u);
            __syncthreads();
            k = s_claim;
            __syncthreads();                         // read by all before the next claim
        } else {
            k = next;
            next += step;
        }
        if (k >= seg_len) break;
        const uint32_t tile = seg_begin + k;
        const int i = find_replica(desc, count, tile);
        const GroupDesc d = desc[i];
        if (s >= d.n) continue;                      // this replica has done its sweeps
        const uint32_t model = model_of<MASK>(d.model);
        if (model != 0u && i != cur) {
            __syncthreads();                         // every wave is done with the old table
            if ((MASK & kMaskBC) && model == 1u) {
                dev::load_bc_table(lds.bc, bc_tables + (size_t)d.tab * 96u);
            } else if constexpr (kLut) {
                const LutRec* rec = luts + d.tab;
                const uint4* src = reinterpret_cast<const uint4*>(rec->buckets);
                uint4* dst = reinterpret_cast<uint4*>(lds.lut.b);
                for (uint32_t k = threadIdx.x; k < (uint32_t)dev::kLutBuckets / 2; k += blockDim.x) dst[k] = src[k];
                if (threadIdx.x < 16) lds.lut.T[threadIdx.x] = rec->T[threadIdx.x];
                __syncthreads();
            }
            cur = i;
        }
        const uint32_t L = d.L;
        const uint32_t t = d.t0 + s;
        const uint32_t g = (tile - d.tile_begin) * 256u + threadIdx.x;
        const size_t plane_words = (size_t)L * (L >> (model == 2u ? 6 : 4));
        uint32_t* own = d.plane0 + (COLOR ? plane_words : 0);
        const uint32_t* oth = d.plane0 + (COLOR ? 0 : plane_words);
        if ((MASK & kMaskLut) && model == 2u) {
            if constexpr (kLut) {
                const uint32_t Q = L >> 8;
                const uint32_t q = g % Q, y0 = (g / Q) * d.rows;
                const LutRec* rec = luts + d.tab;
                const uint32_t T8 = __builtin_amdgcn_readfirstlane(rec->T[8]);
                const uint32_t kmax = __builtin_amdgcn_readfirstlane(rec->kmax);
                if (y0 < L)
                    dev::band_update_lut<0, COLOR>(own, oth, L, d.rows, q, y0, t, d.k0, d.k1, 0u, lds.lut.b,
                                                   lds.lut.T, T8, kmax);
            }
        } else {
            const uint32_t Q = L >> 6;
            const uint32_t q = g % Q, y0 = (g / Q) * d.rows;
            // the thresholds feed scalar operands of the acceptance compares
            const uint32_t T4 = __builtin_amdgcn_readfirstlane(d.T4);
            const uint32_t T8 = __builtin_amdgcn_readfirstlane(d.T8);
            // (a replica's block indices fit 32 bits: L <= 2^17)
            if (y0 < L) {
                const bool wave_rows = (Q & 63u) == 0u;   // the tile's waves each hold one band
                if ((MASK & kMaskBC) && model == 1u) {
                    if (wave_rows)
                        dev::band_update_wave<1, true, COLOR>(own, oth, L, d.rows, q, y0, t, d.k0, d.k1, T4, T8,
                                                              lds.bc.e);
                    else
                        dev::band_update<1, 0, COLOR>(own, oth, L, d.rows, q, y0, t, d.k0, d.k1, 0u, T4, T8,
                                                      lds.bc.e);
                } else if (MASK & kMaskIsing) {
                    if (wave_rows)
                        dev::band_update_wave<0, true, COLOR>(own, oth, L, d.rows, q, y0, t, d.k0, d.k1, T4, T8,
                                                              lds.bc.e);
                    else
                        dev::band_update<0, 0, COLOR>(own, oth, L, d.rows, q, y0, t, d.k0, d.k1, 0u, T4, T8,
                                                      lds.bc.e);
                }
            }
        }
    }
    // every workgroup of the eighth has made its one failed claim when the
    // count of those done reaches its size: no claim is left to come
    if (claim && threadIdx.x == 0 && atomicAdd(&ctr[8 + part], 1u) == step - 1u) {
        atomicExch(&ctr[part], 0u);
        atomicExch(&ctr[8 + part], 0u);
    }
}

// Bucket tables of the 1-bit replicas: block (b, r) writes 256 buckets of replica r.
__global__ __launch_bounds__(256) void group_lut_bucket_kernel(const LutRec* __restrict__ luts)
{
    const LutRec* rec = luts + blockIdx.y;
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= (uint32_t)dev::kLutBuckets) return;
    const uint64_t A = dev::lut_bucket_addend(rec->T, rec->kmax, b);
    rec->buckets[b] = make_uint2((uint32_t)A, (uint32_t)(A >> 32));
}

template <int MASK>
void launch_mask(int color, dim3 grid, hipStream_t st, const GroupDesc* desc, int count, const uint2* tabs,
                 const LutRec* luts, uint32_t total, uint32_t s, const uint32_t* sbase, uint32_t* ctr)
{
    if (color == 0)
        hipLaunchKernelGGL((group_half_kernel<MASK, 0>), grid, dim3(256), 0, st, desc, count, tabs, luts, total, s,
                           sbase, ctr);
    else
        hipLaunchKernelGGL((group_half_kernel<MASK, 1>), grid, dim3(256), 0, st, desc, count, tabs, luts, total, s,
                           sbase, ctr);
}

}  // namespace

hipError_t launch_group_half(int mask, int color, const GroupDesc* desc, int count, uint32_t total, uint32_t grid,
                             const uint2* bc_tables, const LutRec* luts, uint32_t s, const uint32_t* sbase,
                             uint32_t* ctr, hipStream_t st)
{
    if (count <= 0 || total == 0 || grid == 0) return hipSuccess;
    const dim3 g(grid);
    if (grid >= total || (grid & 7u) != 0) ctr = nullptr;       // one workgroup per tile: nothing to claim
    switch (mask) {
    case kMaskIsing: launch_mask<kMaskIsing>(color, g, st, desc, count, bc_tables, luts, total, s, sbase, ctr); break;
    case kMaskBC: launch_mask<kMaskBC>(color, g, st, desc, count, bc_tables, luts, total, s, sbase, ctr); break;
    case kMaskLut: launch_mask<kMaskLut>(color, g, st, desc, count, bc_tables, luts, total, s, sbase, ctr); break;
    case kMaskIsing | kMaskBC:
        launch_mask<kMaskIsing | kMaskBC>(color, g, st, desc, count, bc_tables, luts, total, s, sbase, ctr);
        break;
    default:
        // any mix holding 1-bit replicas
        launch_mask<kMaskIsing | kMaskBC | kMaskLut>(color, g, st, desc, count, bc_tables, luts, total, s, sbase, ctr);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_group_lut_buckets(const LutRec* luts, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(group_lut_bucket_kernel, dim3(dev::kLutBuckets / 256, (uint32_t)n), dim3(256), 0, st, luts);
    return hipGetLastError();
}

}  // namespace mcl
