/*
 * mcl.h -- C ABI of the MI355X (gfx950) library for the checkerboard
 * Metropolis sweep of the 2D Ising and Blume-Capel models and the
 * measurements taken while the lattice relaxes after a quench
 * (Bisson et al., arXiv:2502.18624).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an int status: MCL_OK (0) or a negative MCL_E*
 *    code; nothing throws across the ABI.  mcl_strerror() names a code and
 *    mcl_last_hip_error() returns the HIP error behind the last MCL_EHIP.
 *  - Units J = k_B = 1 (section 3.2 states the Ising flip probabilities as
 *    e^{-4 beta} and e^{-8 beta}); beta = 1/T.  The energy of eq. (BC) is
 *    E = -B + D Q with the integer sums returned by measure(); for the
 *    Ising model (eq. IM) E = -B.
 *  - The lattice is L x L, periodic, site (x, y) with x the fast axis; its
 *    colour is (x + y) & 1 (checkerboard decomposition, section 3.1) and a
 *    sweep updates colour 0, then colour 1.  L must be a multiple of 64
 *    (of 256 for MCL_ISING_LUT), at least 64 and at most 2^20.
 *  - Randomness is counter-based Philox4x32-10 keyed by the 64-bit seed and
 *    addressed by (sweep t, colour, logical site), so results do not depend
 *    on storage layout, batching or launch shape: every lattice is
 *    bit-reproducible.  Counter words, per stream:
 *      accept draw  : k = (y L + x) >> 1; ctr = (k>>2 lo, k>>2 hi, t, c),
 *                     output word k & 3
 *      proposal bit : ctr = (k>>7 lo, k>>7 hi, t, 2 + c), bit k & 31 of
 *                     output word (k >> 5) & 3               (Blume-Capel)
 *      initial draw : n = y L + x; ctr = (n>>2 lo, n>>2 hi, 0, 4), word n & 3
 *  - Acceptance is integer: a move raising the energy by dE > 0 is accepted
 *    iff u < floor(2^32 exp(-beta dE)) (clamped to 2^32 - 1), u the accept
 *    draw; dE <= 0 is always accepted.
 *  - Device memory is owned by the caller: lattice_init() receives one
 *    device buffer of at least mcl_query_bytes() bytes and keeps a
 *    non-owning pointer to it until lattice_free().  Handles are owned by
 *    the library.  Host buffers passed in are owned by the caller and only
 *    read/written during the call.
 *  - Work is queued on the caller's HIP stream (hipStream_t passed as
 *    void*; NULL = the null stream).  sweep() and group_sweep() are
 *    asynchronous; measure(), lattice_read*() and lattice_write()
 *    synchronise that stream before returning.
 *  - One handle must not be used from two threads at once; distinct
 *    handles are independent.
 */
#ifndef MCL_H
#define MCL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcl_lattice mcl_lattice;

/* Models: eq. (IM), spins +-1; eq. (BC), spins -1/0/+1 with crystal field D;
 * MCL_ISING_LUT: eq. (IM) with 1-bit cells and the table-driven random bits
 * of section 3.2 (see mcl_lut_table).  MCL_ISING and MCL_BC store 4-bit
 * cells; MCL_ISING_LUT stores 1-bit cells and needs L a multiple of 256. */
enum { MCL_ISING = 0, MCL_BC = 1, MCL_ISING_LUT = 2 };

/* Initial states.  RANDOM is the T = infinity sample that a quench starts
 * from (section 1): Ising s = +1 iff w < 2^31, Blume-Capel
 * s = floor(3 w / 2^32) - 1, w the initial draw.  ZERO is Blume-Capel only. */
enum { MCL_INIT_RANDOM = 0, MCL_INIT_UP = 1, MCL_INIT_DOWN = 2, MCL_INIT_ZERO = 3 };

/* Correlation modes of measure() (section 3.3).
 *   FULL     : every distance 0..L/2 from every site.
 *   PROTOCOL : every site for r <= 2R = 32; one source per R x R square
 *              (x = y = 0 mod 16) for 32 < r <= r_c(t) and for the
 *              log-spaced distances floor(2^{x/32}) > r_c(t) up to L/2, with
 *              r_c(t) = max{256, floor(g(L) sqrt(t) + 0.5)} and
 *              g(L) = 6 sqrt(ln(L / 2^16) / 3.3^2 + 1).  L a power of two. */
enum { MCL_CORR_NONE = 0, MCL_CORR_FULL = 1, MCL_CORR_PROTOCOL = 2 };

enum {
    MCL_OK = 0,
    MCL_EMODEL = -1,    /* unknown model */
    MCL_EL = -2,        /* L not a multiple of 64 (256 for MCL_ISING_LUT), < 64 or > 2^20 (or PROTOCOL with L not 2^k) */
    MCL_EBETA = -3,     /* beta NaN or negative (beta = +inf is allowed) */
    MCL_ED = -4,        /* D NaN or infinite (Blume-Capel) */
    MCL_EINIT = -5,     /* unknown init state, or ZERO with the Ising model */
    MCL_ENOMEM = -6,    /* dev_bytes smaller than mcl_query_bytes() */
    MCL_ERANGE = -7,    /* the sweep counter t would pass 2^32 - 1; bad window */
    MCL_EHIP = -8,      /* a HIP call failed: see mcl_last_hip_error() */
    MCL_EARG = -9,      /* NULL pointer, negative count, unknown mode */
    MCL_EBUFSZ = -10,   /* caller buffer too small; the needed size is reported */
    MCL_ESPINS = -11,   /* lattice_write() got a value outside the model's spins */
    MCL_ESCRATCH = -12  /* group_sweep_noalloc(): the call exceeds its fixed workspace */
};

/* Output of measure().  The caller owns the arrays r, Cx, Cy, nsrc (r_cap
 * entries each; they may be NULL when corr_mode is MCL_CORR_NONE). */
typedef struct mcl_measure_out {
    int64_t B;          /* sum over sites of s(x,y) [s(x+1,y) + s(x,y+1)] */
    int64_t M;          /* sum of s */
    int64_t Q;          /* sum of s^2 */
    int64_t t;          /* sweeps completed */
    int64_t counts[3];  /* number of spins equal to -1, 0, +1 */
    int64_t invalid;    /* stored cells that hold no spin value; 0 unless corrupted */
    int32_t* r;         /* out: distances */
    int64_t* Cx;        /* out: sum over sources p of s(p) s(p + r e_x) */
    int64_t* Cy;        /* out: sum over sources p of s(p) s(p + r e_y) */
    int64_t* nsrc;      /* out: number of sources at each distance */
    int32_t r_cap;      /* in: capacity of the four arrays */
    int32_t n_r;        /* out: number of distances (also set on MCL_EBUFSZ) */
    int64_t sd[9];      /* out: sd[k] = number of sites with sigma h = k - 4, h the sum of
                         * the four neighbours: the histogram behind the Schwinger-Dyson
                         * check of section 4 (eq. SDI), whose right-hand side is
                         * sum_k sd[k] exp(-2 beta (k - 4)) / L^2 */
} mcl_measure_out;

/* Device bytes lattice_init() needs for an L x L lattice of `model`: two
 * colour planes of 4-bit cells (L^2 / 2 bytes; L^2 / 8 for 1-bit cells)
 * plus measurement scratch and a 256-byte control block. */
int mcl_query_bytes(int model, int64_t L, int64_t* dev_bytes);

/* Create a handle and write the initial state (section 1: quench
 * from a high temperature; see MCL_INIT_*).  dev_mem: caller-owned device
 * buffer of dev_bytes >= mcl_query_bytes(); hip_stream: stream for all of
 * this handle's work.  The sweep counter t starts at 0. */
int lattice_init(mcl_lattice** out, int model, int64_t L, uint64_t seed, int init_state,
                 void* dev_mem, int64_t dev_bytes, void* hip_stream);

/* n checkerboard sweeps (section 3.1: colour 0, then colour 1)
 * of single-spin Metropolis updates (section 1) at inverse temperature beta
 * and crystal field D (finite; ignored for Ising).  Ising: a spin with 3 aligned
 * neighbours flips with probability e^{-4 beta}, with 4 with e^{-8 beta},
 * otherwise always (section 3.2).  Blume-Capel: the proposal is one of the
 * two other values, chosen by the proposal bit (0: next value cyclically in
 * -1,0,+1; 1: the one after), accepted by Metropolis on eq. (BC).
 * Asynchronous on the handle's stream; advances t by n.
 * Lattices of up to 2^24 cells run calls of 32 sweeps or more as replays of
 * an executable HIP graph of 32 sweeps, captured on first use for each
 * (beta, D) (up to four per handle, destroyed by lattice_free) on a
 * library stream of default priority; the sweep index then comes from a
 * word of the handle's device buffer.  The lattices are the same either
 * way.  The environment variable MCL_SWEEP_GRAPH=0 (never) or 1 (at any
 * size) overrides the size rule; it is read on each call.  While the
 * caller captures the handle's stream into a graph of its own, sweep()
 * queues plain launches, which carry absolute sweep indices: each replay of
 * the caller's graph repeats the same t values (t advances once, when the
 * call is captured).  Errors: MCL_EARG
 * (n < 0), MCL_EBETA, MCL_ED, MCL_ERANGE (t + n > 2^32), MCL_EHIP. */
int sweep(mcl_lattice* h, int64_t n, double beta, double D);

/* B, M, Q, spin counts, the sigma h histogram (out->sd) and, if corr_mode !=
 * NONE, the correlation sums along both axes at the distances of the mode
 * for the current t (section 3.3).  Synchronous (waits for the handle's
 * stream, so it must not be captured into a graph).  MCL_EBUFSZ if r_cap <
 * needed (out->n_r then holds the needed size); MCL_EL for the protocol mode
 * with L not a power of two.  The x-correlation of the sampled sources keeps
 * rows in LDS; the environment variable MCL_SX_LDS_BUDGET (bytes, read at
 * every call) lowers its budget below the 160 KiB of a workgroup, which
 * changes the launch shape only, never the result. */
int measure(mcl_lattice* h, int corr_mode, mcl_measure_out* out);

/* Distances measure() would use for (mode, L, t); returns their number, or
 * MCL_EBUFSZ (with *n_needed set) if cap is too small or r is NULL;
 * MCL_EARG for an unknown mode, L < 2 or t < 0; MCL_EL for the protocol
 * with L not a power of two. */
int mcl_rset(int corr_mode, int64_t L, int64_t t, int32_t* r, int32_t cap, int32_t* n_needed);

/* The acceptance thresholds sweep() uses.  Ising: thr[0] = floor(2^32
 * e^{-4 beta}), thr[1] = floor(2^32 e^{-8 beta}), always[] unused.
 * Blume-Capel: 54 entries indexed ((s+1)*2 + b)*9 + (h+4); always[i] = 1
 * where dE <= 0.  dE = -h (s' - s) + D (s'^2 - s^2) in double, that order.
 * Errors: MCL_EMODEL, MCL_EBETA, MCL_ED (Blume-Capel with D NaN or
 * infinite), MCL_EARG, MCL_EBUFSZ (cap < 2, or < 54 for Blume-Capel). */
int mcl_thresholds(int model, double beta, double D, uint32_t* thr, uint8_t* always, int32_t cap);

/* Table of MCL_ISING_LUT (section 3.2): with p = exp(-4 beta) and each of
 * 4 pattern bits set independently with probability p, T[k] =
 * floor(2^32 * C_k), C_k the probability of the patterns 0 .. k-1 summed in
 * that order in double (T[0] = 0; T[k] may be 2^32).  A 32-bit draw u picks
 * the pattern max{k : T[k] <= u}; bit j belongs to in-colour site 4g + j of
 * group g.  Two streams per group g (e = 0: exp4, e = 1: ANDed with exp4
 * into exp8): ctr = (g>>2 lo, g>>2 hi, t, 8 + 2c + e), output word g & 3.
 * A site flips always with at most 2 aligned neighbours, iff its exp4 bit
 * with 3, iff its exp8 bit with 4.  Errors: MCL_EBETA, MCL_EARG (T16 NULL). */
int mcl_lut_table(double beta, uint64_t* T16);

/* Copy the lattice to host memory as L*L int8 spins, row-major [y][x].
 * Synchronous.  Used for parity checks and checkpoints.  MCL_EARG on NULL. */
int lattice_read(mcl_lattice* h, int8_t* host_spins);

/* Window [x0, x0+w) x [y0, y0+hgt) (periodic) as w*hgt int8 spins, row-major.
 * Synchronous.  MCL_ERANGE unless 0 <= x0, y0 < L and 1 <= w, hgt <= L. */
int lattice_read_window(mcl_lattice* h, int64_t x0, int64_t y0, int64_t w, int64_t hgt,
                        int8_t* host_spins);

/* Raw colour planes (both, plane 0 first, in the device layout): L*L/2
 * bytes for 4-bit cells, L*L/8 for 1-bit cells; MCL_EBUFSZ if bytes is
 * smaller.  For checkpoints of large lattices.  The write takes the cells
 * as they are (a cell that holds no spin value is counted by measure() as
 * invalid) and sets the sweep counter t (MCL_ERANGE unless 0 <= t <= 2^32). */
int lattice_read_packed(mcl_lattice* h, void* host, int64_t bytes);
int lattice_write_packed(mcl_lattice* h, const void* host, int64_t bytes, int64_t t);

/* Restore: L*L int8 spins and the sweep counter t.  MCL_ESPINS for a value
 * the model does not have (0 for Ising), MCL_ERANGE unless 0 <= t <= 2^32. */
int lattice_write(mcl_lattice* h, const int8_t* host_spins, int64_t t);

/* Handle state; NULL outputs are skipped.  MCL_EARG if h is NULL. */
int lattice_info(const mcl_lattice* h, int* model, int64_t* L, uint64_t* seed, int64_t* t);

/* Batched path: advance `count` independent lattices (any mix of
 * models, sizes, beta and D) by n[i] sweeps each.  Replicas advance sweep by
 * sweep together.  Every lattice of L <= 2^17 with n[i] > 0 goes into one
 * launch per colour per sweep that covers all of them, all three models
 * alike (or, with the split_models tuning, one launch per model and
 * colour): a persistent grid walks a list of tiles of 256 threads, each
 * tile one band of rows of one replica, so a replica's parameters are
 * wave-uniform.  Larger lattices fill the GPU alone and are swept one per
 * launch within the call.  All lattices must use the stream of hs[0], and
 * no two entries with n[i] > 0 may share device memory (the same handle
 * twice, or handles on overlapping buffers), which would race: MCL_EARG
 * otherwise, before anything is queued.  Every lattice ends bit-identical
 * to n[i] sweep() calls on it alone, whatever the tuning.  The launches of
 * a call shape seen before are replayed from an executable HIP graph of
 * graph_sweeps sweeps (captured on the second sighting; not while the
 * caller captures the stream).  MCL_ERANGE if a launch would need more than
 * 2^24 workgroups.  The library keeps a few small workspaces of its own
 * (descriptors, pinned staging, captured graphs), allocated on first use
 * and grown when a larger group arrives; they are never freed. */
int group_sweep(mcl_lattice* const* hs, int count, const int64_t* n,
                const double* beta, const double* D);

/* group_sweep() for callers that cannot allocate memory: code that must
 * not call hipMalloc (tight serving loops, harnesses that forbid it).  Same
 * arguments, checks, results and errors as group_sweep(): every lattice
 * ends bit-identical to n[i] sweep() calls on it alone.  It allocates
 * nothing -- no device or pinned memory, no graph, no event, no host heap:
 *  - the call's descriptor image is staged in a fixed host array and copied
 *    (hipMemcpyAsync on the lattices' stream) into a fixed device array of
 *    1 MiB that each GPU the library runs on holds until the process ends;
 *    the array's address and two events per device are taken once, at
 *    set-up (lattice_init(), or the first call on that device);
 *  - the batched launches are plain ones (no captured graph), and lattices
 *    larger than 2^17 are swept by plain launches too.
 * Limits: at most 4096 entries, and an image of at most 1 MiB, which holds
 * at least 1200 batched replicas of any mix (a Blume-Capel replica takes
 * 832 bytes, an Ising one 64, a 1-bit one 144): MCL_ESCRATCH beyond, before
 * anything is queued.  The fixed arrays keep the last call's image.  Calls
 * on one GPU share them, so the library orders them: a call's copy waits
 * for the previous call's launches on that GPU (whatever their stream),
 * and the host array is rewritten only after the previous call's copy has
 * run (the host may block for that).  Calls from several threads are
 * serialised by a lock.  Not for use inside a stream capture of the
 * caller's (the copy reads pageable host memory).  Runs on the current
 * device, which must be the lattices' device. */
int group_sweep_noalloc(mcl_lattice* const* hs, int count, const int64_t* n,
                        const double* beta, const double* D);

/* Tuning of group_sweep, process-wide; chosen by the package's autotuner.
 * Results never depend on it.
 *   rows_log2L[k] : band height (rows per thread: 8, 16, 32 or 64) for
 *                   lattices with 2^k <= L < 2^(k+1);
 *   use_graph     : replay repeated call shapes from captured graphs;
 *   largest_first : order each launch's tile list by decreasing L (else
 *                   call order);
 *   wg_per_cu     : persistent grid of wg_per_cu workgroups per compute unit
 *                   (1..32), or 0 for one workgroup per tile;
 *   split_models  : one launch per model and colour instead of one per colour
 *                   (each launch then holds one model's code path and
 *                   register budget);
 *   graph_sweeps  : sweeps per captured graph (1..64). */
typedef struct mcl_group_tuning {
    int32_t rows_log2L[21];
    int32_t use_graph;
    int32_t largest_first;
    int32_t wg_per_cu;
    int32_t split_models;
    int32_t graph_sweeps;
} mcl_group_tuning;
int mcl_group_tuning_get(mcl_group_tuning* out);
int mcl_group_tuning_set(const mcl_group_tuning* in);   /* MCL_EARG on a value out of range */

/* Release a handle (does not free the caller's device memory).  Waits for
 * the handle's stream first, so the buffer is free for reuse on return,
 * then destroys the handle's graphs. */
int lattice_free(mcl_lattice* h);

const char* mcl_strerror(int code);
int mcl_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MCL_H */
