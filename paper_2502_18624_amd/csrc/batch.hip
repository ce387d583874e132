// Batched half-sweep: many independent lattices -- any mix of
// sizes, temperatures, crystal fields and seeds -- advance in one launch per
// model and colour.  Each workgroup belongs to exactly one replica (its task
// range is padded to whole workgroups), so the replica's parameters are
// wave-uniform and the per-thread work is the one-lattice band update of
// sweep_device.h: every lattice ends bit-identical to its own sweeps.
#include "internal.h"
#include "sweep_device.h"

namespace mcl {
namespace {

// Replica of workgroup `wg`: last descriptor with wg_begin <= wg.
__device__ __forceinline__ int find_replica(const GroupDesc* __restrict__ desc, int count, uint32_t wg)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].wg_begin <= wg) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int MODEL, int COLOR>
__global__ __launch_bounds__(256) void group_half_kernel(const GroupDesc* __restrict__ desc, int count,
                                                         const uint2* __restrict__ tables, uint32_t s)
{
    __shared__ dev::BCLds s_tab;
    const int i = find_replica(desc, count, blockIdx.x);
    const GroupDesc d = desc[i];
    if (s >= d.n) return;
    if (MODEL == 1) dev::load_bc_table(s_tab, tables + (size_t)d.bc * 96u);
    const uint32_t L = d.L;
    const uint32_t Q = L >> 6;
    const uint32_t g = (blockIdx.x - d.wg_begin) * blockDim.x + threadIdx.x;
    const uint32_t q = g % Q;
    const uint32_t band = g / Q;
    const uint32_t y0 = band * d.rows;
    if (y0 >= L) return;
    const size_t plane_words = (size_t)L * (L >> 4);
    uint32_t* own = d.plane0 + (COLOR ? plane_words : 0);
    const uint32_t* oth = d.plane0 + (COLOR ? 0 : plane_words);
    // the thresholds feed scalar operands of the acceptance compares
    const uint32_t T4 = __builtin_amdgcn_readfirstlane(d.T4);
    const uint32_t T8 = __builtin_amdgcn_readfirstlane(d.T8);
    const uint32_t t = d.t0 + s;
    uint32_t hu;
    const int hm = dev::counter_mode(d.hi0 != 0, ((uint64_t)y0 * (L >> 1) + 32u * q) >> 2,
                                     ((uint64_t)(y0 + d.rows - 1) * (L >> 1) + 32u * q + 31u) >> 2, hu);
    if (hm == 0)
        dev::band_update<MODEL, 0, COLOR>(own, oth, L, d.rows, q, y0, t, d.k0, d.k1, 0u, T4, T8, s_tab.e);
    else if (hm == 1)
        dev::band_update<MODEL, 1, COLOR>(own, oth, L, d.rows, q, y0, t, d.k0, d.k1, hu, T4, T8, s_tab.e);
    else
        dev::band_update<MODEL, 2, COLOR>(own, oth, L, d.rows, q, y0, t, d.k0, d.k1, 0u, T4, T8, s_tab.e);
}

}  // namespace

hipError_t launch_group_half(int model, int color, const GroupDesc* desc, int count, uint32_t total_wgs,
                             const uint2* tables, uint32_t s, hipStream_t st)
{
    if (count <= 0 || total_wgs == 0) return hipSuccess;
    const dim3 grid(total_wgs), blk(256);
    if (model == 0) {
        if (color == 0) hipLaunchKernelGGL((group_half_kernel<0, 0>), grid, blk, 0, st, desc, count, tables, s);
        else hipLaunchKernelGGL((group_half_kernel<0, 1>), grid, blk, 0, st, desc, count, tables, s);
    } else {
        if (color == 0) hipLaunchKernelGGL((group_half_kernel<1, 0>), grid, blk, 0, st, desc, count, tables, s);
        else hipLaunchKernelGGL((group_half_kernel<1, 1>), grid, blk, 0, st, desc, count, tables, s);
    }
    return hipGetLastError();
}

}  // namespace mcl
