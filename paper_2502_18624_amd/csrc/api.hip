// C ABI of the library (declared in include/mcl.h): handles, argument
// checks, host-side acceptance tables and correlation distances, and the
// plain one-lattice-per-launch sweep driver.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/mcl.h"
#include "internal.h"

struct mcl_lattice {
    int model;
    int64_t L;
    uint64_t seed;
    int64_t t;
    mcl::Geom g;
    int64_t* acc;        // device: kAccSlots int64
    int32_t* rdev;       // device: distances, rcap entries
    int64_t* Cx;         // device: rcap entries
    int64_t* Cy;         // device: rcap entries
    uint32_t* tbits;     // device: T bits of the sampled columns (measure scratch)
    void* lutb;          // device: bucket table of the 1-bit mode (1-bit lattices only)
    uint32_t* tdev;      // device: sweep index at the start of a replayed graph
    int64_t rcap;
    hipStream_t stream;
    // measure() of 1-bit lattices: the sampled y pass runs on `side` (created
    // at the first measurement with sampled distances), between the events
    // `fork` (the T bits are written) and `join` (before the results are read)
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // executable graphs of kGraphSweeps sweeps, one per (beta, D) in use
    struct SweepGraph {
        double beta, D;
        hipGraphExec_t exec;
    };
    std::vector<SweepGraph> graphs;
};

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return MCL_EHIP;
}

#define MCL_HIP(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_);     \
    } while (0)

int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

bool valid_model(int model) { return model == MCL_ISING || model == MCL_BC || model == MCL_ISING_LUT; }

bool valid_L(int model, int64_t L)
{
    const int64_t q = model == MCL_ISING_LUT ? 256 : 64;
    return L >= q && (L % q) == 0 && L <= (int64_t(1) << 20);
}

int cell_bits(int model) { return model == MCL_ISING_LUT ? 1 : 4; }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

struct Layout {
    int64_t planes, acc, rlist, cx, cy, tbits, ctl, lutb, total, rcap;
};

Layout layout_of(int model, int64_t L)
{
    Layout lay;
    lay.rcap = L / 2 + 1;
    int64_t off = 0;
    lay.planes = off;
    off += align256(L * L * cell_bits(model) / 8);
    lay.acc = off;
    off += align256(mcl::kAccSlots * 8);
    lay.rlist = off;
    off += align256(lay.rcap * 4);
    lay.cx = off;
    off += align256(lay.rcap * 8);
    lay.cy = off;
    off += align256(lay.rcap * 8);
    lay.tbits = off;
    off += align256(mcl::tbits_bytes(model, L));
    lay.ctl = off;
    off += 256;
    lay.lutb = off;
    if (model == MCL_ISING_LUT) off += mcl::kLutBucketBytes;
    lay.total = off;
    return lay;
}

// floor(2^32 exp(-beta dE)) clamped to 2^32 - 1, for dE > 0 (the integer
// form of the Metropolis acceptance probability).
uint32_t threshold_of(double beta, double dE)
{
    const double scaled = std::ldexp(std::exp(-beta * dE), 32);
    if (scaled >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)std::floor(scaled);
}

// Table of the 1-bit mode (section 3.2): cumulative probabilities of the
// 4-bit patterns in index order, each bit set with p = e^{-4 beta}.
void lut_table64(double beta, uint64_t T[16])
{
    const double p = std::exp(-4.0 * beta);
    double cum = 0.0;
    for (int k = 0; k < 16; ++k) {
        T[k] = (uint64_t)std::floor(std::ldexp(cum, 32));
        double prob = 1.0;
        for (int j = 0; j < 4; ++j) prob *= ((k >> j) & 1) ? p : (1.0 - p);
        cum += prob;
    }
}

mcl::LutTable lut_device_table(double beta)
{
    uint64_t T[16];
    lut_table64(beta, T);
    mcl::LutTable d;
    d.kmax = 0;
    for (int k = 0; k < 16; ++k) {
        d.T[k] = T[k] > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)T[k];
        if (T[k] <= 0xFFFFFFFFull) d.kmax = (uint32_t)k;
    }
    return d;
}

void ising_thresholds(double beta, uint32_t& T4, uint32_t& T8)
{
    T4 = threshold_of(beta, 4.0);   // three aligned neighbours: dE = 4
    T8 = threshold_of(beta, 8.0);   // four aligned neighbours:  dE = 8
}

// Blume-Capel: entry ((n * 2) + b) * 9 + hsum with n = s + 1, hsum = h + 4;
// proposal s' = ((n + 1 + b) mod 3) - 1; dE of eq. (BC) with J = 1.
void bc_table(double beta, double D, mcl::BCTable& tb)
{
    for (int n = 0; n < 3; ++n)
        for (int b = 0; b < 2; ++b)
            for (int hsum = 0; hsum < 9; ++hsum) {
                const int s = n - 1, h = hsum - 4;
                const int s2 = ((n + 1 + b) % 3) - 1;
                const double dE = (double)(-h * (s2 - s)) + D * (double)(s2 * s2 - s * s);
                const int idx = (n * 2 + b) * 9 + hsum;
                if (dE <= 0.0) {
                    tb.always[idx] = 1;
                    tb.thr[idx] = 0;
                } else {
                    tb.always[idx] = 0;
                    tb.thr[idx] = threshold_of(beta, dE);
                }
            }
}

// Correlation distances (section 3.3); returns them sorted ascending with
// the count of leading "every source" distances in n_all.
std::vector<int32_t> distances(int mode, int64_t L, int64_t t, int32_t* n_all)
{
    std::vector<int32_t> r;
    const int64_t half = L / 2;
    if (mode == MCL_CORR_FULL) {
        for (int64_t v = 0; v <= half; ++v) r.push_back((int32_t)v);
        if (n_all) *n_all = (int32_t)r.size();
        return r;
    }
    const int64_t R2 = 32;
    const double g = 6.0 * std::sqrt(std::log((double)L / 65536.0) / (3.3 * 3.3) + 1.0);
    int64_t rc = (int64_t)std::floor(g * std::sqrt((double)t) + 0.5);
    if (rc < 256) rc = 256;
    for (int64_t v = 0; v <= std::min(half, R2); ++v) r.push_back((int32_t)v);
    if (n_all) *n_all = (int32_t)r.size();
    for (int64_t v = R2 + 1; v <= std::min(half, rc); ++v) r.push_back((int32_t)v);
    int64_t lg = 0;
    while ((int64_t(1) << lg) < L) ++lg;
    const int64_t xmax = 32 * (lg - 1);
    for (int64_t x = 1; x <= xmax; ++x) {
        const int64_t d = (int64_t)std::floor(std::pow(2.0, (double)x / 32.0));
        if (d > rc && d <= half && (r.empty() || r.back() != d)) r.push_back((int32_t)d);
    }
    return r;
}

int check_params(const mcl_lattice* h, double beta, double D)
{
    if (std::isnan(beta) || beta < 0.0) return MCL_EBETA;
    // an infinite D would make dE = D (s'^2 - s^2) undefined (infinity times
    // zero) for the moves s -> -s
    if (h->model == MCL_BC && !std::isfinite(D)) return MCL_ED;
    return MCL_OK;
}

// Cell i of a row (W words) as a spin, for 4-bit cells (n - 1) or 1-bit
// cells (bit ? +1 : -1).
int8_t cell_to_spin(const uint32_t* row, int64_t i, int cb)
{
    if (cb == 1) return ((row[i >> 5] >> (i & 31)) & 1u) ? (int8_t)1 : (int8_t)-1;
    return (int8_t)((int)((row[i >> 3] >> (4 * (i & 7))) & 0xFu) - 1);
}

void spin_to_cell(uint32_t* row, int64_t i, int s, int cb)
{
    if (cb == 1) {
        if (s > 0) row[i >> 5] |= 1u << (i & 31);
        return;
    }
    row[i >> 3] |= (uint32_t)(s + 1) << (4 * (i & 7));
}

// ---------------------------------------------------------------------------
// Batched path.
// ---------------------------------------------------------------------------
// Lattices up to this size go into the batched launches; larger ones fill
// the GPU on their own and are swept one per launch.
constexpr int64_t kGroupMaxL = int64_t(1) << 17;
// Entries of one group_sweep_noalloc call (its fixed host workspaces).
constexpr int kNoAllocEntries = 4096;

mcl_group_tuning default_tuning()
{
    mcl_group_tuning t;
    for (int k = 0; k < 21; ++k) t.rows_log2L[k] = k >= 12 ? 32 : 16;
    t.use_graph = 1;
    t.largest_first = 1;
    t.wg_per_cu = 0;
    t.split_models = 0;
    t.graph_sweeps = 32;
    return t;
}

bool valid_tuning(const mcl_group_tuning& t)
{
    for (int k = 0; k < 21; ++k) {
        const int r = t.rows_log2L[k];
        if (r != 8 && r != 16 && r != 32 && r != 64) return false;
    }
    return t.wg_per_cu >= 0 && t.wg_per_cu <= 32 && t.graph_sweeps >= 1 && t.graph_sweeps <= 64 &&
           (t.use_graph == 0 || t.use_graph == 1) && (t.largest_first == 0 || t.largest_first == 1) &&
           (t.split_models == 0 || t.split_models == 1);
}

std::mutex g_group_mu;
mcl_group_tuning g_tuning = default_tuning();

int log2_floor(int64_t v)
{
    int k = 0;
    while ((int64_t(1) << (k + 1)) <= v) ++k;
    return k;
}

// Blume-Capel table in the kernel's LDS order: 96 entries indexed
// (n * 2 + b) * 16 + neighbour-cell-sum, x = threshold, y = always.
void bc_lds_table(double beta, double D, uint32_t* out /* 192 words */)
{
    mcl::BCTable tb;
    bc_table(beta, D, tb);
    for (int i = 0; i < 96; ++i) {
        const int key = i >> 4, sj = i & 15;
        uint32_t thr = 0, alw = 0;
        if (key < 6 && sj < 9) {
            const int idx = key * 9 + sj;        // ((n * 2 + b) * 9 + sum)
            thr = tb.thr[idx];
            alw = tb.always[idx] ? 1u : 0u;
        }
        out[2 * i] = thr;
        out[2 * i + 1] = alw;
    }
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int compute_units(int dev)
{
    static std::map<int, int> cache;
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cache[dev] = cus;
    return cus;
}

// The launches of one batched call and the device image they read:
// descriptors (launch by launch), Blume-Capel tables, 1-bit records, and a
// 256-byte block holding the word a captured graph adds its sweep offset to
// (word 0) and the tile-claim counters of persistent launches (words 16 to
// 31), all uploaded as zero.
struct GroupLaunch {
    int mask;          // models in the launch (kMask*)
    size_t first;      // its first descriptor
    int count;
    uint32_t total;    // tiles
    uint32_t grid;     // workgroups (a multiple of 8)
};
struct GroupImage {
    GroupLaunch launches[3];   // one per model, or one for all
    int nlaunch = 0;
    size_t ndesc = 0, nbc = 0, nlut = 0;
    size_t off_bc = 0, off_lut = 0, off_s = 0, bytes = 0;
    int64_t nmax = 0;
};

// Replicas of the batched launches: n > 0 and L <= kGroupMaxL.
bool batched(const mcl_lattice* h, int64_t n) { return n > 0 && h->L <= kGroupMaxL; }

// Plan the call (launches, tiles, grid) into `img`; when `host` is given,
// also write the image there (it must hold img.bytes).  `order` is room for
// `count` entry indices.  Allocates nothing.  MCL_ERANGE if a launch would
// need more than 2^24 workgroups or 2^32 tiles.
int group_layout(mcl_lattice* const* hs, int count, const int64_t* n, const double* beta, const double* D,
                 const mcl_group_tuning& tun, int cus, GroupImage& img, void* host, int* order)
{
    img = GroupImage();
    for (int i = 0; i < count; ++i)
        if (batched(hs[i], n[i])) {
            img.nmax = std::max(img.nmax, n[i]);
            img.ndesc++;
            img.nbc += hs[i]->model == MCL_BC;
            img.nlut += hs[i]->model == MCL_ISING_LUT;
        }
    img.off_bc = align_up(img.ndesc * sizeof(mcl::GroupDesc), 256);
    img.off_lut = align_up(img.off_bc + img.nbc * 96 * sizeof(uint2), 256);
    img.off_s = align_up(img.off_lut + img.nlut * sizeof(mcl::LutRec), 256);
    img.bytes = img.off_s + 256;
    char* base = (char*)host;
    // the sweep-offset word and the claim counters start at 0
    if (base) std::memset(base + img.off_s, 0, 256);
    mcl::GroupDesc* hd = (mcl::GroupDesc*)base;
    uint32_t* htab = base ? (uint32_t*)(base + img.off_bc) : nullptr;
    mcl::LutRec* hlut = base ? (mcl::LutRec*)(base + img.off_lut) : nullptr;
    size_t k = 0, nb = 0, nl = 0;
    for (int m = 0; m < (tun.split_models ? 3 : 1); ++m) {
        int cnt = 0;
        for (int i = 0; i < count; ++i)
            if (batched(hs[i], n[i]) && (!tun.split_models || hs[i]->model == m)) order[cnt++] = i;
        if (cnt == 0) continue;
        // decreasing L, call order among equal L (an in-place sort on the pair)
        if (tun.largest_first)
            std::sort(order, order + cnt,
                      [&](int a, int b) { return hs[a]->L != hs[b]->L ? hs[a]->L > hs[b]->L : a < b; });
        GroupLaunch ln{0, k, cnt, 0, 0};
        uint64_t tiles = 0;
        for (int j = 0; j < cnt; ++j) {
            const int i = order[j];
            const mcl_lattice* h = hs[i];
            const uint32_t rows = (uint32_t)tun.rows_log2L[log2_floor(h->L)];
            const int64_t threads = h->g.Q * (h->L / rows);
            ln.mask |= h->model == MCL_ISING ? mcl::kMaskIsing : h->model == MCL_BC ? mcl::kMaskBC : mcl::kMaskLut;
            if (base) {
                mcl::GroupDesc d;
                std::memset(&d, 0, sizeof(d));
                d.plane0 = h->g.plane0;
                d.L = (uint32_t)h->L;
                d.rows = rows;
                d.t0 = (uint32_t)h->t;
                d.n = (uint32_t)n[i];
                d.k0 = (uint32_t)h->seed;
                d.k1 = (uint32_t)(h->seed >> 32);
                d.tile_begin = (uint32_t)tiles;
                d.model = (uint32_t)h->model;
                if (h->model == MCL_ISING) {
                    ising_thresholds(beta[i], d.T4, d.T8);
                } else if (h->model == MCL_BC) {
                    d.tab = (uint32_t)nb;
                    bc_lds_table(beta[i], D[i], htab + nb * 192);
                } else {
                    d.tab = (uint32_t)nl;
                    const mcl::LutTable lt = lut_device_table(beta[i]);
                    mcl::LutRec r;
                    std::memset(&r, 0, sizeof(r));
                    r.buckets = (uint2*)h->lutb;
                    std::memcpy(r.T, lt.T, sizeof(r.T));
                    r.kmax = lt.kmax;
                    hlut[nl] = r;
                }
                hd[k] = d;
            }
            nb += h->model == MCL_BC;
            nl += h->model == MCL_ISING_LUT;
            ++k;
            tiles += (uint64_t)((threads + 255) / 256);
        }
        if (tiles >= (uint64_t(1) << 32)) return MCL_ERANGE;
        ln.total = (uint32_t)tiles;
        // one workgroup per tile, or a persistent grid of wg_per_cu per CU;
        // a multiple of 8 either way (one share per XCD)
        uint64_t grid = (tiles + 7) / 8 * 8;
        if (tun.wg_per_cu > 0) grid = std::min<uint64_t>(grid, (uint64_t)cus * tun.wg_per_cu / 8 * 8);
        grid = std::max<uint64_t>(grid, 8);
        if (grid > (uint64_t(1) << 24)) return MCL_ERANGE;
        ln.grid = (uint32_t)grid;
        img.launches[img.nlaunch++] = ln;
    }
    return MCL_OK;
}

// Launches of sweeps [s0, s0 + k) of a planned call on stream st, the
// image at `dev` (sbase: device word added to s, or nullptr).
hipError_t group_launches(const GroupImage& img, const void* dev, int64_t s0, int64_t k, const uint32_t* sbase,
                          hipStream_t st)
{
    const char* b = (const char*)dev;
    const mcl::GroupDesc* desc = (const mcl::GroupDesc*)b;
    const uint2* tabs = (const uint2*)(b + img.off_bc);
    const mcl::LutRec* luts = (const mcl::LutRec*)(b + img.off_lut);
    uint32_t* ctr = (uint32_t*)(b + img.off_s) + 16;
    for (int64_t s = s0; s < s0 + k; ++s)
        for (int c = 0; c < 2; ++c)
            for (int j = 0; j < img.nlaunch; ++j) {
                const GroupLaunch& ln = img.launches[j];
                const hipError_t e = mcl::launch_group_half(ln.mask, c, desc + ln.first, ln.count, ln.total, ln.grid,
                                                            tabs, luts, (uint32_t)s, sbase, ctr, st);
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}

// Work of a planned call whose image is already on its way to `dev` on
// stream st: the 1-bit bucket tables, then the sweeps as plain launches.
hipError_t group_plain(const GroupImage& img, const void* dev, hipStream_t st)
{
    hipError_t e = mcl::launch_group_lut_buckets((const mcl::LutRec*)((const char*)dev + img.off_lut), (int)img.nlut,
                                                 st);
    if (e != hipSuccess) return e;
    return group_launches(img, dev, 0, img.nmax, nullptr, st);
}

// A staging slot: pinned host buffer and device buffer for one call's
// image, and an event recorded after the call's last launch.  A slot is
// reused only after that event completed, so at most one call per slot is
// in flight and neither buffer is overwritten while a copy or kernel reads
// it.  Graphs captured against the slot's device buffer live with the slot.
struct SlotGraph {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
    uint64_t last_use;
};
struct Slot {
    void* host = nullptr;
    void* dev = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    std::vector<SlotGraph> graphs;
};
constexpr int kSlots = 4;
constexpr size_t kSlotGraphs = 8;
struct DeviceSlots {
    Slot slot[kSlots];
    int next = 0;
    std::vector<std::vector<uint64_t>> seen;      // recent call shapes (a graph is captured on a repeat)
};
std::map<int, DeviceSlots> g_slots;
uint64_t g_graph_clock = 0;

// Graph capture is not allowed on the null stream, which is where a caller
// on PyTorch's default stream queues its work; such calls capture and
// replay on a library stream (default priority) fenced by events.
struct CaptureStream {
    hipStream_t stream = nullptr;
    hipEvent_t in = nullptr, out = nullptr;
};
std::map<int, CaptureStream> g_capture;

void destroy_graphs(Slot& sl)
{
    for (auto& g : sl.graphs) (void)hipGraphExecDestroy(g.exec);        // best effort: the slot is idle
    sl.graphs.clear();
}

// The executable graph of k sweeps of the planned call on slot sl (sweep
// index *sdev + i, then *sdev += k), captured on stream gs if absent.
int slot_graph(Slot& sl, const GroupImage& img, int64_t k, hipStream_t gs, const std::vector<uint64_t>& key,
               hipGraphExec_t* out)
{
    for (auto& g : sl.graphs)
        if (g.key == key) {
            g.last_use = ++g_graph_clock;
            *out = g.exec;
            return MCL_OK;
        }
    uint32_t* sdev = (uint32_t*)((char*)sl.dev + img.off_s);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    MCL_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed));
    hipError_t le = group_launches(img, sl.dev, 0, k, sdev, gs);
    if (le == hipSuccess) le = mcl::launch_set_word(sdev, (uint32_t)k, true, gs);
    const hipError_t ce = hipStreamEndCapture(gs, &graph);
    if (ce == hipSuccess && le != hipSuccess) (void)hipGraphDestroy(graph);
    if (le != hipSuccess) return hip_fail(le);
    if (ce != hipSuccess) return hip_fail(ce);
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);                       // the executable graph keeps what it needs
    if (ie != hipSuccess) return hip_fail(ie);
    if (sl.graphs.size() >= kSlotGraphs) {
        // least recently used; the slot is idle (its last call completed), so is the graph
        auto lru = std::min_element(sl.graphs.begin(), sl.graphs.end(),
                                    [](const SlotGraph& a, const SlotGraph& b) { return a.last_use < b.last_use; });
        (void)hipGraphExecDestroy(lru->exec);
        sl.graphs.erase(lru);
    }
    sl.graphs.push_back({key, exec, ++g_graph_clock});
    *out = exec;
    return MCL_OK;
}

int group_run(mcl_lattice* const* hs, int count, const int64_t* n, const double* beta, const double* D)
{
    std::lock_guard<std::mutex> lk(g_group_mu);
    const mcl_group_tuning tun = g_tuning;
    hipStream_t stream = hs[0]->stream;
    int devid = 0;
    MCL_HIP(hipGetDevice(&devid));
    GroupImage img;
    std::vector<int> order((size_t)count);
    int rc = group_layout(hs, count, n, beta, D, tun, compute_units(devid), img, nullptr, order.data());
    if (rc) return rc;
    if (img.nmax == 0) return MCL_OK;

    DeviceSlots& ds = g_slots[devid];
    Slot& sl = ds.slot[ds.next];
    ds.next = (ds.next + 1) % kSlots;
    if (sl.pending) {
        MCL_HIP(hipEventSynchronize(sl.done));
        sl.pending = false;
    }
    if (!sl.done) MCL_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    if (sl.cap < img.bytes) {
        destroy_graphs(sl);                               // they read the old device buffer
        if (sl.host) MCL_HIP(hipHostFree(sl.host));
        if (sl.dev) MCL_HIP(hipFree(sl.dev));
        sl.host = sl.dev = nullptr;
        sl.cap = 0;
        const size_t cap = std::max<size_t>(img.bytes * 2, 64 * 1024);
        MCL_HIP(hipHostMalloc(&sl.host, cap, hipHostMallocDefault));
        MCL_HIP(hipMalloc(&sl.dev, cap));
        sl.cap = cap;
    }
    rc = group_layout(hs, count, n, beta, D, tun, compute_units(devid), img, sl.host, order.data());
    if (rc) return rc;
    MCL_HIP(hipMemcpyAsync(sl.dev, sl.host, img.bytes, hipMemcpyHostToDevice, stream));

    // graph replays for a shape seen before (and not inside a capture of the caller's)
    const int64_t K = std::min<int64_t>(tun.graph_sweeps, img.nmax);
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(stream, &cst) != hipSuccess || cst != hipStreamCaptureStatusNone;
    bool use_graph = tun.use_graph && !capturing && img.nmax >= 2;
    std::vector<uint64_t> key;
    if (use_graph) {
        key = {(uint64_t)(uintptr_t)sl.dev, (uint64_t)K, (uint64_t)img.off_bc, (uint64_t)img.off_lut,
               (uint64_t)img.off_s};
        for (int j = 0; j < img.nlaunch; ++j) {
            const GroupLaunch& ln = img.launches[j];
            key.insert(key.end(), {(uint64_t)ln.mask, (uint64_t)ln.first, (uint64_t)ln.count, (uint64_t)ln.total,
                                   (uint64_t)ln.grid});
        }
        // a shape is captured the second time it is seen: one-off shapes run plain
        std::vector<uint64_t> shape(key.begin() + 1, key.end());
        const bool known = std::any_of(sl.graphs.begin(), sl.graphs.end(),
                                       [&](const SlotGraph& g) { return g.key == key; });
        const bool seen = std::find(ds.seen.begin(), ds.seen.end(), shape) != ds.seen.end();
        if (!seen) {
            ds.seen.push_back(shape);
            if (ds.seen.size() > 16) ds.seen.erase(ds.seen.begin());
        }
        use_graph = known || seen;
    }
    if (!use_graph) {
        MCL_HIP(group_plain(img, sl.dev, stream));
    } else {
        MCL_HIP(mcl::launch_group_lut_buckets((const mcl::LutRec*)((const char*)sl.dev + img.off_lut), (int)img.nlut,
                                              stream));
        hipStream_t gs = stream;
        CaptureStream* cs = nullptr;
        if (stream == nullptr) {
            cs = &g_capture[devid];
            if (!cs->stream) {
                MCL_HIP(hipStreamCreateWithFlags(&cs->stream, hipStreamNonBlocking));
                MCL_HIP(hipEventCreateWithFlags(&cs->in, hipEventDisableTiming));
                MCL_HIP(hipEventCreateWithFlags(&cs->out, hipEventDisableTiming));
            }
            gs = cs->stream;
            MCL_HIP(hipEventRecord(cs->in, stream));
            MCL_HIP(hipStreamWaitEvent(gs, cs->in, 0));
        }
        hipGraphExec_t exec = nullptr;
        rc = slot_graph(sl, img, K, gs, key, &exec);
        if (rc) return rc;
        const int64_t reps = img.nmax / K;
        for (int64_t r = 0; r < reps; ++r) MCL_HIP(hipGraphLaunch(exec, gs));
        if (reps * K < img.nmax)
            MCL_HIP(group_launches(img, sl.dev, reps * K, img.nmax - reps * K, nullptr, gs));
        if (cs) {
            MCL_HIP(hipEventRecord(cs->out, gs));
            MCL_HIP(hipStreamWaitEvent(stream, cs->out, 0));
        }
    }
    MCL_HIP(hipEventRecord(sl.done, stream));
    sl.pending = true;
    return MCL_OK;
}

// Acceptance parameters of one sweep() call.
struct SweepParams {
    uint32_t T4 = 0, T8 = 0;     // Ising
    mcl::BCTable tb{};           // Blume-Capel
    mcl::LutTable tab{};         // 1-bit Ising
};

// The launches of n sweeps of h on stream s, sweep indices t, t + 1, ...
// (plus the device word *tbase when given).
hipError_t launch_sweeps(const mcl_lattice* h, const SweepParams& p, int64_t n, uint32_t t, const uint32_t* tbase,
                         hipStream_t s)
{
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 2; ++c) {
            const uint32_t ti = t + (uint32_t)i;
            hipError_t e;
            if (h->model == MCL_ISING_LUT) {
                e = mcl::launch_lut_half(h->g, c, ti, tbase, h->seed, p.tab, h->lutb, s);
            } else {
                mcl::HalfSweepArgs a{};
                a.color = c;
                a.t = ti;
                a.tbase = tbase;
                a.seed = h->seed;
                a.T4 = p.T4;
                a.T8 = p.T8;
                a.bc = &p.tb;
                e = h->model == MCL_ISING ? mcl::launch_ising_half(h->g, a, s) : mcl::launch_bc_half(h->g, a, s);
            }
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

// Small lattices replay a captured graph of kGraphSweeps sweeps.  Kernels
// in a graph follow each other sooner than separate launches (a trivial
// kernel: 2.0 against 2.8 us on the null stream); measured on half-sweeps
// this saves 0.1-0.4 us each (2-7%) up to L = 2^12 and nothing from 2^13 on,
// where a half-sweep lasts long enough to hide the dispatch of the next.
// The environment variable MCL_SWEEP_GRAPH = 0 or 1 turns the replay off or
// on at any size.
constexpr int64_t kGraphSweeps = 32;
constexpr int64_t kGraphMaxCells = int64_t(1) << 24;   // L <= 2^12

bool use_sweep_graph(const mcl_lattice* h)
{
    // a stream that the caller is capturing gets plain launches: no graph
    // of the library's own is captured or launched inside the caller's
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(h->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
    if (const char* e = std::getenv("MCL_SWEEP_GRAPH")) {
        if (e[0] == '0') return false;
        if (e[0] == '1') return true;
    }
    return h->L * h->L <= kGraphMaxCells;
}

std::mutex g_sweep_capture_mu;
std::map<int, hipStream_t> g_sweep_capture;        // per device, default priority, only ever captures

// The executable graph of h for (beta, D), captured on first use: sweeps
// *tdev + i for i < kGraphSweeps, then *tdev += kGraphSweeps.
int sweep_graph(mcl_lattice* h, double beta, double D, const SweepParams& p, hipGraphExec_t* out)
{
    const double key_D = h->model == MCL_BC ? D : 0.0;
    for (const auto& sg : h->graphs)
        if (sg.beta == beta && sg.D == key_D) {
            *out = sg.exec;
            return MCL_OK;
        }
    int dev = 0;
    MCL_HIP(hipGetDevice(&dev));
    hipGraph_t graph = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_sweep_capture_mu);
        hipStream_t& cs = g_sweep_capture[dev];
        if (!cs) MCL_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        MCL_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        hipError_t le = launch_sweeps(h, p, kGraphSweeps, 0u, h->tdev, cs);
        if (le == hipSuccess) le = mcl::launch_set_word(h->tdev, (uint32_t)kGraphSweeps, true, cs);
        const hipError_t ce = hipStreamEndCapture(cs, &graph);
        if (ce == hipSuccess && le != hipSuccess) (void)hipGraphDestroy(graph);
        if (le != hipSuccess) return hip_fail(le);
        if (ce != hipSuccess) return hip_fail(ce);
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);                           // the executable graph keeps what it needs
    if (ie != hipSuccess) return hip_fail(ie);
    if (h->graphs.size() >= 4) {
        // the oldest graph may still be queued on the lattice's stream
        MCL_HIP(hipStreamSynchronize(h->stream));
        (void)hipGraphExecDestroy(h->graphs.front().exec);
        h->graphs.erase(h->graphs.begin());
    }
    h->graphs.push_back({beta, key_D, exec});
    *out = exec;
    return MCL_OK;
}

// sweep() after its argument checks; allow_graph = false queues plain
// launches only (no graph is captured or created).
int sweep_checked(mcl_lattice* h, int64_t n, double beta, double D, bool allow_graph)
{
    if (n == 0) return MCL_OK;
    SweepParams p{};
    if (h->model == MCL_ISING_LUT) {
        p.tab = lut_device_table(beta);
        MCL_HIP(mcl::launch_lut_buckets(p.tab, h->lutb, h->stream));
    } else if (h->model == MCL_ISING) {
        ising_thresholds(beta, p.T4, p.T8);
    } else {
        bc_table(beta, D, p.tb);
    }
    int64_t done = 0;
    if (allow_graph && n >= kGraphSweeps && use_sweep_graph(h)) {
        hipGraphExec_t exec = nullptr;
        const int rc = sweep_graph(h, beta, D, p, &exec);
        if (rc) return rc;
        MCL_HIP(mcl::launch_set_word(h->tdev, (uint32_t)h->t, false, h->stream));
        for (; done + kGraphSweeps <= n; done += kGraphSweeps) MCL_HIP(hipGraphLaunch(exec, h->stream));
    }
    if (done < n) MCL_HIP(launch_sweeps(h, p, n - done, (uint32_t)(h->t + done), nullptr, h->stream));
    h->t += n;
    return MCL_OK;
}

// ---------------------------------------------------------------------------
// Argument checks and the lattices outside the batched launches, shared by
// group_sweep and group_sweep_noalloc.
// ---------------------------------------------------------------------------
using Span = std::pair<uintptr_t, uintptr_t>;

// `spans` is room for `count` entries.  Allocates nothing.
int group_check(mcl_lattice* const* hs, int count, const int64_t* n, const double* beta, const double* D, Span* spans)
{
    if (count < 0 || (count > 0 && (!hs || !n || !beta || !D))) return MCL_EARG;
    for (int i = 0; i < count; ++i) {
        if (!hs[i] || n[i] < 0) return MCL_EARG;
        if (hs[i]->stream != hs[0]->stream) return MCL_EARG;
        const int pc = check_params(hs[i], beta[i], D[i]);
        if (pc) return pc;
        if (hs[i]->t + n[i] > (int64_t(1) << 32)) return MCL_ERANGE;
    }
    // entries that do work must not share device memory: their updates would
    // run concurrently on the same cells (or on a 1-bit replica's bucket table)
    int ns = 0;
    for (int i = 0; i < count; ++i)
        if (n[i] > 0) {
            const uintptr_t a = (uintptr_t)hs[i]->g.plane0;
            spans[ns++] = Span(a, a + (uintptr_t)layout_of(hs[i]->model, hs[i]->L).total);
        }
    std::sort(spans, spans + ns);
    for (int k = 1; k < ns; ++k)
        if (spans[k].first < spans[k - 1].second) return MCL_EARG;
    return MCL_OK;
}

// After the batched launches: advance their counters, and sweep each
// lattice larger than kGroupMaxL on its own (it fills the GPU alone).
int group_finish(mcl_lattice* const* hs, int count, const int64_t* n, const double* beta, const double* D,
                 bool allow_graph)
{
    for (int i = 0; i < count; ++i) {
        if (batched(hs[i], n[i])) {
            hs[i]->t += n[i];
        } else if (n[i] > 0) {
            const int rc = sweep_checked(hs[i], n[i], beta[i], D[i], allow_graph);
            if (rc) return rc;
        }
    }
    return MCL_OK;
}

// ---------------------------------------------------------------------------
// Non-allocating batched path (group_sweep_noalloc).  The call's image
// (descriptors, Blume-Capel tables, 1-bit records) is staged in a fixed host
// array and copied into `scratch`, a fixed device array: each GPU holds its
// own copy of it for the life of the process.  In host code the array's
// name is no device address; its address on a device comes from
// hipGetSymbolAddress, taken once per device at set-up (lattice_init, or
// the first call on that device) and used for every copy and launch.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = size_t(1) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct NoAllocDevice {
    void* ptr = nullptr;          // this device's copy of scratch
    hipEvent_t copied = nullptr;  // after the last copy out of the host image
    hipEvent_t done = nullptr;    // after the last call's launches
    bool pending = false;
};
NoAllocDevice g_noalloc[kMaxDevices];
alignas(256) unsigned char g_noalloc_host[kNoAllocBytes];
int g_noalloc_order[kNoAllocEntries];
Span g_noalloc_spans[kNoAllocEntries];
int g_noalloc_last = -1;          // device of the last copy out of g_noalloc_host

// Set-up of device devid (current); the caller holds g_group_mu.
int noalloc_setup(int devid)
{
    if (devid < 0 || devid >= kMaxDevices) return MCL_EARG;
    NoAllocDevice& st = g_noalloc[devid];
    if (st.ptr) return MCL_OK;
    void* ptr = nullptr;
    MCL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!st.copied) MCL_HIP(hipEventCreateWithFlags(&st.copied, hipEventDisableTiming));
    if (!st.done) MCL_HIP(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    (void)compute_units(devid);   // fills its cache here rather than in a call
    st.ptr = ptr;
    return MCL_OK;
}

// The batched launches of a checked call, with no allocation of any kind;
// the caller holds g_group_mu.
int group_run_noalloc(mcl_lattice* const* hs, int count, const int64_t* n, const double* beta, const double* D)
{
    mcl_group_tuning tun = g_tuning;
    hipStream_t stream = hs[0]->stream;
    int devid = 0;
    MCL_HIP(hipGetDevice(&devid));
    int rc = noalloc_setup(devid);
    if (rc) return rc;
    NoAllocDevice& st = g_noalloc[devid];
    GroupImage img;
    rc = group_layout(hs, count, n, beta, D, tun, compute_units(devid), img, nullptr, g_noalloc_order);
    if (rc) return rc;
    if (img.nmax == 0) return MCL_OK;
    if (img.bytes > kNoAllocBytes) return MCL_ESCRATCH;
    // the host image is free once the copy of the last call (on any device) has run
    if (g_noalloc_last >= 0 && g_noalloc[g_noalloc_last].pending) {
        MCL_HIP(hipEventSynchronize(g_noalloc[g_noalloc_last].copied));
        g_noalloc[g_noalloc_last].pending = false;
    }
    rc = group_layout(hs, count, n, beta, D, tun, compute_units(devid), img, g_noalloc_host, g_noalloc_order);
    if (rc) return rc;
    // the device image is rewritten only after the launches of the previous
    // call on this device, whatever stream they were queued on
    MCL_HIP(hipStreamWaitEvent(stream, st.done, 0));
    MCL_HIP(hipMemcpyAsync(st.ptr, g_noalloc_host, img.bytes, hipMemcpyHostToDevice, stream));
    MCL_HIP(hipEventRecord(st.copied, stream));
    st.pending = true;
    g_noalloc_last = devid;
    MCL_HIP(group_plain(img, st.ptr, stream));
    MCL_HIP(hipEventRecord(st.done, stream));
    return MCL_OK;
}

}  // namespace

extern "C" {

const char* mcl_strerror(int code)
{
    switch (code) {
    case MCL_OK: return "ok";
    case MCL_EMODEL: return "unknown model";
    case MCL_EL: return "L must be a multiple of 64 (256 for 1-bit cells), at most 2^20 (a power of two for the protocol)";
    case MCL_EBETA: return "beta must be >= 0 (NaN rejected)";
    case MCL_ED: return "D must be finite";
    case MCL_EINIT: return "unknown initial state for this model";
    case MCL_ENOMEM: return "device buffer smaller than mcl_query_bytes()";
    case MCL_ERANGE: return "value out of range (sweep counter or window)";
    case MCL_EHIP: return "HIP runtime error (see mcl_last_hip_error)";
    case MCL_EARG: return "invalid argument";
    case MCL_EBUFSZ: return "caller buffer too small";
    case MCL_ESPINS: return "spin value not allowed for this model";
    case MCL_ESCRATCH:
        return "group_sweep_noalloc: more than 4096 entries, or a batched image above its fixed 1 MiB workspace "
               "(at least 1200 replicas of any mix)";
    default: return "unknown error";
    }
}

int mcl_last_hip_error(void) { return g_last_hip; }

int mcl_query_bytes(int model, int64_t L, int64_t* dev_bytes)
{
    if (!valid_model(model)) return MCL_EMODEL;
    if (!valid_L(model, L)) return MCL_EL;
    if (!dev_bytes) return MCL_EARG;
    *dev_bytes = layout_of(model, L).total;
    return MCL_OK;
}

int mcl_lut_table(double beta, uint64_t* T16)
{
    if (std::isnan(beta) || beta < 0.0) return MCL_EBETA;
    if (!T16) return MCL_EARG;
    lut_table64(beta, T16);
    return MCL_OK;
}

int mcl_thresholds(int model, double beta, double D, uint32_t* thr, uint8_t* always, int32_t cap)
{
    if (model != MCL_ISING && model != MCL_BC) return MCL_EMODEL;
    if (std::isnan(beta) || beta < 0.0) return MCL_EBETA;
    if (!thr) return MCL_EARG;
    if (model == MCL_ISING) {
        if (cap < 2) return MCL_EBUFSZ;
        ising_thresholds(beta, thr[0], thr[1]);
        return MCL_OK;
    }
    if (!std::isfinite(D)) return MCL_ED;
    if (cap < 54 || !always) return cap < 54 ? MCL_EBUFSZ : MCL_EARG;
    mcl::BCTable tb;
    bc_table(beta, D, tb);
    for (int i = 0; i < 54; ++i) {
        thr[i] = tb.thr[i];
        always[i] = (uint8_t)tb.always[i];
    }
    return MCL_OK;
}

int mcl_rset(int corr_mode, int64_t L, int64_t t, int32_t* r, int32_t cap, int32_t* n_needed)
{
    if (corr_mode != MCL_CORR_FULL && corr_mode != MCL_CORR_PROTOCOL) return MCL_EARG;
    if (L < 2 || t < 0) return MCL_EARG;
    if (corr_mode == MCL_CORR_PROTOCOL && !is_pow2(L)) return MCL_EL;
    const std::vector<int32_t> d = distances(corr_mode, L, t, nullptr);
    if (n_needed) *n_needed = (int32_t)d.size();
    if ((int64_t)d.size() > cap || !r) return MCL_EBUFSZ;
    std::memcpy(r, d.data(), d.size() * sizeof(int32_t));
    return (int)d.size();
}

int lattice_init(mcl_lattice** out, int model, int64_t L, uint64_t seed, int init_state, void* dev_mem,
                 int64_t dev_bytes, void* hip_stream)
{
    if (!out || !dev_mem) return MCL_EARG;
    *out = nullptr;
    if (!valid_model(model)) return MCL_EMODEL;
    if (!valid_L(model, L)) return MCL_EL;
    if (init_state < MCL_INIT_RANDOM || init_state > MCL_INIT_ZERO) return MCL_EINIT;
    if (init_state == MCL_INIT_ZERO && model != MCL_BC) return MCL_EINIT;
    const Layout lay = layout_of(model, L);
    if (dev_bytes < lay.total) return MCL_ENOMEM;
    if (((uintptr_t)dev_mem & 255) != 0) return MCL_EARG;
    mcl_lattice* h = new (std::nothrow) mcl_lattice;
    if (!h) return MCL_EARG;
    char* base = (char*)dev_mem;
    h->model = model;
    h->L = L;
    h->seed = seed;
    h->t = 0;
    h->g.L = L;
    h->g.cb = cell_bits(model);
    h->g.W = h->g.cb == 1 ? L / 64 : L / 16;
    h->g.Q = h->g.cb == 1 ? L / 256 : L / 64;
    h->g.plane0 = (uint32_t*)(base + lay.planes);
    h->acc = (int64_t*)(base + lay.acc);
    h->rdev = (int32_t*)(base + lay.rlist);
    h->Cx = (int64_t*)(base + lay.cx);
    h->Cy = (int64_t*)(base + lay.cy);
    h->tbits = (uint32_t*)(base + lay.tbits);
    h->lutb = model == MCL_ISING_LUT ? (void*)(base + lay.lutb) : nullptr;
    h->tdev = (uint32_t*)(base + lay.ctl);
    h->rcap = lay.rcap;
    h->stream = (hipStream_t)hip_stream;
    {
        // set-up of group_sweep_noalloc on this device (best effort: that
        // entry point repeats it and reports a failure itself)
        std::lock_guard<std::mutex> lk(g_group_mu);
        int devid = 0;
        if (hipGetDevice(&devid) == hipSuccess) (void)noalloc_setup(devid);
    }
    const hipError_t e = model == MCL_ISING_LUT ? mcl::launch_init1(h->g, init_state, seed, h->stream)
                                                : mcl::launch_init(h->g, model, init_state, seed, h->stream);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e);
    }
    *out = h;
    return MCL_OK;
}

int lattice_free(mcl_lattice* h)
{
    if (!h) return MCL_EARG;
    // work queued on the lattice (sweeps, graph replays) may still be running:
    // let it finish before the caller can reuse the buffer or the graphs go
    (void)hipStreamSynchronize(h->stream);                 // best effort: the handle goes either way
    for (const auto& sg : h->graphs) (void)hipGraphExecDestroy(sg.exec);
    if (h->side) (void)hipStreamDestroy(h->side);           // idle: measure() joins it before returning
    if (h->fork) (void)hipEventDestroy(h->fork);
    if (h->join) (void)hipEventDestroy(h->join);
    delete h;
    return MCL_OK;
}

int lattice_info(const mcl_lattice* h, int* model, int64_t* L, uint64_t* seed, int64_t* t)
{
    if (!h) return MCL_EARG;
    if (model) *model = h->model;
    if (L) *L = h->L;
    if (seed) *seed = h->seed;
    if (t) *t = h->t;
    return MCL_OK;
}

int sweep(mcl_lattice* h, int64_t n, double beta, double D)
{
    if (!h || n < 0) return MCL_EARG;
    const int pc = check_params(h, beta, D);
    if (pc) return pc;
    if (h->t + n > (int64_t(1) << 32)) return MCL_ERANGE;
    return sweep_checked(h, n, beta, D, true);
}

int measure(mcl_lattice* h, int corr_mode, mcl_measure_out* out)
{
    if (!h || !out) return MCL_EARG;
    if (corr_mode != MCL_CORR_NONE && corr_mode != MCL_CORR_FULL && corr_mode != MCL_CORR_PROTOCOL) return MCL_EARG;
    if (corr_mode == MCL_CORR_PROTOCOL && !is_pow2(h->L)) return MCL_EL;
    std::vector<int32_t> r;
    int32_t n_all = 0;
    if (corr_mode != MCL_CORR_NONE) {
        r = distances(corr_mode, h->L, h->t, &n_all);
        out->n_r = (int32_t)r.size();
        if ((int64_t)r.size() > out->r_cap) return MCL_EBUFSZ;
        if (!out->r || !out->Cx || !out->Cy || !out->nsrc) return MCL_EARG;
        if ((int64_t)r.size() > h->rcap) return MCL_EBUFSZ;
    } else {
        out->n_r = 0;
    }
    const int nr = (int)r.size();
    MCL_HIP(mcl::launch_zero(h->acc, mcl::kAccSlots, h->stream));
    if (nr > 0) {
        MCL_HIP(hipMemcpyAsync(h->rdev, r.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
        MCL_HIP(mcl::launch_zero(h->Cx, nr, h->stream));
        MCL_HIP(mcl::launch_zero(h->Cy, nr, h->stream));
    }
    const int ns = nr - n_all;                          // sampled distances
    // 4-bit Ising cells with correlations at L >= 4096: the short-distance
    // tiles give B, M, Q, the histogram and the T bits too, so the lattice is
    // read once; cells that hold no spin set acc[14], and then the B/M/Q pass
    // runs after all (below)
    const bool fused = nr > 0 && mcl::bmq_fused(h->g, h->model);
    mcl::SampledArgs sa;
    sa.r = h->rdev + n_all;
    sa.nr = ns;
    sa.Cx = h->Cx + n_all;
    sa.Cy = h->Cy + n_all;
    sa.tbits = h->tbits;
    if (fused) sa.rbits = h->tbits + h->L * mcl::tbits_words(h->L);
    if (ns > 0) {
        // the sampled distances start with a run of consecutive ones (the
        // linear range up to r_c(t)), which the y pass takes apart
        sa.rlin0 = (uint32_t)r[n_all];
        sa.nlin = 1;
        while (sa.nlin < ns && r[n_all + sa.nlin] == r[n_all] + sa.nlin) ++sa.nlin;
    }
    // 1-bit lattices: the sampled y pass, which reads only the T bits and is
    // bound by cache reads, runs on the side stream as soon as the B/M/Q pass
    // has written them, beside the short-distance tiles, which are bound by
    // VALU issue.  For 4-bit cells it overlaps worse (Blume-Capel's tiles hold
    // fewer waves, and the fused Ising path has only the sampled x pass left
    // to run beside it), so there everything stays on the lattice's stream.
    const bool side_y = ns > 0 && h->model == MCL_ISING_LUT;
    if (side_y && !h->side) {
        MCL_HIP(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        MCL_HIP(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming));
        MCL_HIP(hipEventCreateWithFlags(&h->join, hipEventDisableTiming));
    }
    if (!fused) MCL_HIP(mcl::launch_bmq(h->g, h->model, h->acc, ns > 0 ? h->tbits : nullptr, h->stream));
    if (side_y) {
        MCL_HIP(hipEventRecord(h->fork, h->stream));
        MCL_HIP(hipStreamWaitEvent(h->side, h->fork, 0));
        MCL_HIP(mcl::launch_corr_sampled_y(h->g, h->model, sa, h->side));
        MCL_HIP(hipEventRecord(h->join, h->side));
    }
    if (nr > 0) {
        // every-source distances are r = 0 .. n_all - 1 (position j holds r = j)
        const int rshort = std::min(n_all - 1, 32);
        MCL_HIP(mcl::launch_corr_short(h->g, h->model, rshort, h->Cx, h->Cy, fused ? h->acc : nullptr,
                                       fused && ns > 0 ? h->tbits : nullptr, h->stream));
        if (n_all - 1 > 32)
            MCL_HIP(mcl::launch_corr_all(h->g, h->rdev + 33, n_all - 33, h->Cx + 33, h->Cy + 33, h->stream));
        if (ns > 0) {
            MCL_HIP(mcl::launch_corr_sampled_x(h->g, h->model, sa, h->stream));
            if (side_y)
                MCL_HIP(hipStreamWaitEvent(h->stream, h->join, 0));
            else
                MCL_HIP(mcl::launch_corr_sampled_y(h->g, h->model, sa, h->stream));
        }
    }
    int64_t acc[mcl::kAccSlots];
    MCL_HIP(hipMemcpyAsync(acc, h->acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
    if (nr > 0) {
        MCL_HIP(hipMemcpyAsync(out->Cx, h->Cx, nr * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
        MCL_HIP(hipMemcpyAsync(out->Cy, h->Cy, nr * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
    }
    MCL_HIP(hipStreamSynchronize(h->stream));
    if (fused && acc[14] != 0) {
        MCL_HIP(mcl::launch_zero(h->acc, mcl::kAccSlots, h->stream));
        MCL_HIP(mcl::launch_bmq(h->g, h->model, h->acc, nullptr, h->stream));
        MCL_HIP(hipMemcpyAsync(acc, h->acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
        MCL_HIP(hipStreamSynchronize(h->stream));
    }
    out->B = acc[0];
    out->M = acc[1];
    out->Q = acc[2] + acc[3];
    out->counts[0] = acc[3];
    out->counts[1] = acc[4];
    out->counts[2] = acc[2];
    out->invalid = h->L * h->L - acc[2] - acc[3] - acc[4];
    for (int k = 0; k < 9; ++k) out->sd[k] = acc[5 + k];
    out->t = h->t;
    const int64_t all_src = h->L * h->L;
    const int64_t sampled_src = (h->L / 16) * (h->L / 16);
    for (int j = 0; j < nr; ++j) {
        out->r[j] = r[j];
        out->nsrc[j] = (j < n_all) ? all_src : sampled_src;
    }
    return MCL_OK;
}

int lattice_read_packed(mcl_lattice* h, void* host, int64_t bytes)
{
    if (!h || !host) return MCL_EARG;
    const int64_t need = 2 * h->L * h->g.W * 4;
    if (bytes < need) return MCL_EBUFSZ;
    MCL_HIP(hipStreamSynchronize(h->stream));
    MCL_HIP(hipMemcpyAsync(host, h->g.plane0, need, hipMemcpyDeviceToHost, h->stream));
    MCL_HIP(hipStreamSynchronize(h->stream));
    return MCL_OK;
}

int lattice_write_packed(mcl_lattice* h, const void* host, int64_t bytes, int64_t t)
{
    if (!h || !host) return MCL_EARG;
    if (t < 0 || t > (int64_t(1) << 32)) return MCL_ERANGE;
    const int64_t need = 2 * h->L * h->g.W * 4;
    if (bytes < need) return MCL_EBUFSZ;
    MCL_HIP(hipMemcpyAsync(h->g.plane0, host, need, hipMemcpyHostToDevice, h->stream));
    MCL_HIP(hipStreamSynchronize(h->stream));
    h->t = t;
    return MCL_OK;
}

int lattice_read(mcl_lattice* h, int8_t* host_spins)
{
    if (!h || !host_spins) return MCL_EARG;
    const int64_t L = h->L, W = h->g.W;
    std::vector<uint32_t> buf((size_t)(2 * L * W));
    const int rc = lattice_read_packed(h, buf.data(), (int64_t)buf.size() * 4);
    if (rc) return rc;
    for (int64_t y = 0; y < L; ++y)
        for (int64_t x = 0; x < L; ++x) {
            const int c = (int)((x + y) & 1);
            host_spins[y * L + x] = cell_to_spin(buf.data() + (size_t)(c * L * W + y * W), x >> 1, h->g.cb);
        }
    return MCL_OK;
}

int lattice_read_window(mcl_lattice* h, int64_t x0, int64_t y0, int64_t w, int64_t hgt, int8_t* host_spins)
{
    if (!h || !host_spins) return MCL_EARG;
    const int64_t L = h->L, W = h->g.W;
    if (w <= 0 || hgt <= 0 || w > L || hgt > L || x0 < 0 || y0 < 0 || x0 >= L || y0 >= L) return MCL_ERANGE;
    MCL_HIP(hipStreamSynchronize(h->stream));
    std::vector<uint32_t> rows((size_t)(2 * W));
    for (int64_t dy = 0; dy < hgt; ++dy) {
        const int64_t y = (y0 + dy) % L;
        for (int c = 0; c < 2; ++c)
            MCL_HIP(hipMemcpyAsync(rows.data() + c * W, h->g.plane(c) + y * W, W * 4, hipMemcpyDeviceToHost,
                                   h->stream));
        MCL_HIP(hipStreamSynchronize(h->stream));
        for (int64_t dx = 0; dx < w; ++dx) {
            const int64_t x = (x0 + dx) % L;
            const int c = (int)((x + y) & 1);
            host_spins[dy * w + dx] = cell_to_spin(rows.data() + (size_t)(c * W), x >> 1, h->g.cb);
        }
    }
    return MCL_OK;
}

int lattice_write(mcl_lattice* h, const int8_t* host_spins, int64_t t)
{
    if (!h || !host_spins) return MCL_EARG;
    if (t < 0 || t > (int64_t(1) << 32)) return MCL_ERANGE;
    const int64_t L = h->L, W = h->g.W;
    std::vector<uint32_t> buf((size_t)(2 * L * W), 0u);
    for (int64_t y = 0; y < L; ++y)
        for (int64_t x = 0; x < L; ++x) {
            const int s = host_spins[y * L + x];
            const bool ok = (h->model != MCL_BC) ? (s == 1 || s == -1) : (s >= -1 && s <= 1);
            if (!ok) return MCL_ESPINS;
            const int c = (int)((x + y) & 1);
            spin_to_cell(buf.data() + (size_t)(c * L * W + y * W), x >> 1, s, h->g.cb);
        }
    return lattice_write_packed(h, buf.data(), (int64_t)buf.size() * 4, t);
}

int group_sweep(mcl_lattice* const* hs, int count, const int64_t* n, const double* beta, const double* D)
{
    std::vector<Span> spans((size_t)std::max(count, 0));
    int rc = group_check(hs, count, n, beta, D, spans.data());
    if (rc || count == 0) return rc;
    rc = group_run(hs, count, n, beta, D);
    if (rc) return rc;
    return group_finish(hs, count, n, beta, D, true);
}

int group_sweep_noalloc(mcl_lattice* const* hs, int count, const int64_t* n, const double* beta, const double* D)
{
    if (count > kNoAllocEntries) return MCL_ESCRATCH;
    int rc;
    {
        std::lock_guard<std::mutex> lk(g_group_mu);
        rc = group_check(hs, count, n, beta, D, g_noalloc_spans);
        if (rc || count == 0) return rc;
        rc = group_run_noalloc(hs, count, n, beta, D);
    }
    if (rc) return rc;
    return group_finish(hs, count, n, beta, D, false);
}

int mcl_group_tuning_get(mcl_group_tuning* out)
{
    if (!out) return MCL_EARG;
    std::lock_guard<std::mutex> lk(g_group_mu);
    *out = g_tuning;
    return MCL_OK;
}

int mcl_group_tuning_set(const mcl_group_tuning* in)
{
    if (!in || !valid_tuning(*in)) return MCL_EARG;
    std::lock_guard<std::mutex> lk(g_group_mu);
    g_tuning = *in;
    return MCL_OK;
}

}  // extern "C"
