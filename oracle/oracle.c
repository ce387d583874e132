/*
 * CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg load it; the product path
 * never does.  It shares no code with the HIP library.
 *
 * Every routine below is the plain definition, or the method's steps in the
 * order the paper gives them, on an int8 lattice with scalar loops.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As   */
/* Easy as 1, 2, 3", SC'11).  The paper draws its 32-bit uniforms from this  */
/* generator (section 3.2).  State: four 32-bit counter words and a two-word */
/* key.  One round multiplies counter words 0 and 2 by fixed 32-bit          */
/* multipliers, producing 64-bit products, and mixes their halves with the   */
/* other two words and the key; the key is advanced by two Weyl constants     */
/* between rounds.  Ten rounds.                                               */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; round++) {
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        uint32_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        if (round < 9) {            /* key schedule: bump between rounds */
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Counter contract.  The paper names the generator but not how its streams  */
/* are laid out (section 3.2).  Reading: one 64-bit seed per lattice is the  */
/* key (low word first); the counter names the logical site, the sweep t and */
/* the stream, so a draw never depends on how spins are stored.              */
/*   accept draw  : k = (y*L+x)>>1, ctr = (k>>2 lo, k>>2 hi, t, colour),      */
/*                  word k&3                                                 */
/*   proposal bit : ctr = (k>>7 lo, k>>7 hi, t, 2+colour), bit k&31 of word   */
/*                  (k>>5)&3                                                 */
/*   initial draw : n = y*L+x, ctr = (n>>2 lo, n>>2 hi, 0, 4), word n&3       */
/* ------------------------------------------------------------------------ */
static void seed_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

uint32_t ora_accept_draw(uint64_t seed, uint32_t t, int color, uint64_t k)
{
    uint32_t key[2], ctr[4], out[4];
    uint64_t block = k >> 2;
    seed_key(seed, key);
    ctr[0] = (uint32_t)(block & 0xFFFFFFFFu);
    ctr[1] = (uint32_t)(block >> 32);
    ctr[2] = t;
    ctr[3] = (uint32_t)color;
    ora_philox4x32_10(ctr, key, out);
    return out[k & 3];
}

int ora_proposal_bit(uint64_t seed, uint32_t t, int color, uint64_t k)
{
    uint32_t key[2], ctr[4], out[4];
    uint64_t block = k >> 7;
    seed_key(seed, key);
    ctr[0] = (uint32_t)(block & 0xFFFFFFFFu);
    ctr[1] = (uint32_t)(block >> 32);
    ctr[2] = t;
    ctr[3] = (uint32_t)(2 + color);
    ora_philox4x32_10(ctr, key, out);
    return (int)((out[(k >> 5) & 3] >> (k & 31)) & 1u);
}

uint32_t ora_init_draw(uint64_t seed, uint64_t n)
{
    uint32_t key[2], ctr[4], out[4];
    uint64_t block = n >> 2;
    seed_key(seed, key);
    ctr[0] = (uint32_t)(block & 0xFFFFFFFFu);
    ctr[1] = (uint32_t)(block >> 32);
    ctr[2] = 0;
    ctr[3] = 4;
    ora_philox4x32_10(ctr, key, out);
    return out[n & 3];
}

/* ------------------------------------------------------------------------ */
/* Non-uniform random bits (section 3.2).  One 32-bit uniform yields four    */
/* bits, each set with probability p = e^{-4 beta}, by a search in a sorted  */
/* table of 16 entries.  The table's construction is given only in a cited  */
/* reference; reading: entry k is the cumulative probability of the patterns */
/* 0 .. k-1 (pattern bits independent Bernoulli(p)) scaled by 2^32 and      */
/* floored; the search returns the largest k whose entry is <= u, so        */
/* pattern k is drawn with probability (T[k+1] - T[k]) / 2^32.              */
/* Draws: group g = k >> 2 of in-colour sites, stream e, counter             */
/* (g>>2 lo, g>>2 hi, t, 8 + 2 colour + e), output word g & 3; bit j of the  */
/* pattern belongs to site 4g + j.                                          */
/* ------------------------------------------------------------------------ */
void ora_lut_table(double beta, uint64_t T[16])
{
    double p = exp(-4.0 * beta);
    double cum = 0.0;
    int k, j;
    for (k = 0; k < 16; k++) {
        double prob = 1.0;
        T[k] = (uint64_t)floor(ldexp(cum, 32));
        for (j = 0; j < 4; j++)
            prob *= ((k >> j) & 1) ? p : (1.0 - p);
        cum += prob;
    }
}

int ora_lut_lookup(const uint64_t T[16], uint32_t u)
{
    int k, best = 0;
    for (k = 0; k < 16; k++)
        if (T[k] <= (uint64_t)u) best = k;
    return best;
}

uint32_t ora_lut_draw(uint64_t seed, uint32_t t, int color, int e, uint64_t g)
{
    uint32_t key[2], ctr[4], out[4];
    uint64_t block = g >> 2;
    seed_key(seed, key);
    ctr[0] = (uint32_t)(block & 0xFFFFFFFFu);
    ctr[1] = (uint32_t)(block >> 32);
    ctr[2] = t;
    ctr[3] = (uint32_t)(8 + 2 * color + e);
    ora_philox4x32_10(ctr, key, out);
    return out[g & 3];
}

/* ------------------------------------------------------------------------ */
/* Acceptance thresholds.  Metropolis accepts a move that raises the energy  */
/* by dE with probability exp(-beta dE) (section 3.2 states it for the Ising */
/* case: e^{-4 beta} with three aligned neighbours, e^{-8 beta} with four;   */
/* J = k_B = 1).  Reading: the comparison is integer, u < floor(2^32 p)      */
/* with u a 32-bit uniform, p evaluated in IEEE double with the host libm.   */
/* ------------------------------------------------------------------------ */
uint32_t ora_threshold(double beta, double dE)
{
    double p = exp(-beta * dE);
    double scaled = ldexp(p, 32);
    if (scaled >= 4294967295.0)
        return 0xFFFFFFFFu;
    return (uint32_t)floor(scaled);
}

double ora_ising_flip_prob(int aligned, double beta)
{
    /* section 3.2: probability e^{-4 beta} with exactly three aligned
     * neighbours, e^{-8 beta} with four, one otherwise. */
    if (aligned == 3) return ldexp((double)ora_threshold(beta, 4.0), -32);
    if (aligned == 4) return ldexp((double)ora_threshold(beta, 8.0), -32);
    return 1.0;
}

/* Blume-Capel proposal (the paper names Metropolis updates, section 1, but
 * no proposal rule):
 * reading -- propose one of the two other values of {-1,0,+1} uniformly,
 * b = 0 picks the next value cyclically, b = 1 the one after. */
static int bc_propose(int s, int b)
{
    int idx = s + 1;
    return ((idx + 1 + b) % 3) - 1;
}

/* Energy change of s -> s2 under eq. (BC), J = 1, crystal field D,
 * h = sum of the four neighbours; evaluated in exactly this order. */
static double bc_delta_e(int s, int s2, int h, double D)
{
    return (double)(-h * (s2 - s)) + D * (double)(s2 * s2 - s * s);
}

double ora_bc_accept_prob(int s, int h, int b, double beta, double D)
{
    int s2 = bc_propose(s, b);
    double dE = bc_delta_e(s, s2, h, D);
    if (dE <= 0.0) return 1.0;
    return ldexp((double)ora_threshold(beta, dE), -32);
}

/* ------------------------------------------------------------------------ */
/* Initial state: a quench from a high temperature (section 1), i.e. a       */
/* T = infinity sample: Ising +1/-1 with probability 1/2 each; Blume-Capel   */
/* -1/0/+1 uniformly.  Ordered states for tests.                             */
/* ------------------------------------------------------------------------ */
int ora_init(int8_t* s, int model, int64_t L, uint64_t seed, int init_state)
{
    int64_t n, N = L * L;
    if (L < 3) return -1;
    if (model != ORA_ISING && model != ORA_BC && model != ORA_ISING_LUT) return -1;
    if (init_state == ORA_INIT_ZERO && model != ORA_BC) return -1;
    for (n = 0; n < N; n++) {
        int v;
        if (init_state == ORA_INIT_UP) v = 1;
        else if (init_state == ORA_INIT_DOWN) v = -1;
        else if (init_state == ORA_INIT_ZERO) v = 0;
        else {
            uint32_t w = ora_init_draw(seed, (uint64_t)n);
            if (model != ORA_BC)
                v = (w < 0x80000000u) ? 1 : -1;
            else
                v = (int)(((uint64_t)w * 3u) >> 32) - 1;
        }
        s[n] = (int8_t)v;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The sweep.  Checkerboard decomposition (section 3.1): a site's colour is  */
/* (x + y) & 1; one step updates every colour-0 site, then every colour-1    */
/* site, each from its four periodic neighbours (eq. IM / eq. BC).  For even */
/* L sites of one colour only see the other colour, so the order within a    */
/* colour is immaterial; for odd L (allowed here for exact enumeration only) */
/* the sites of a colour are visited in raster order.                        */
/* ------------------------------------------------------------------------ */
static int8_t at(const int8_t* s, int64_t L, int64_t x, int64_t y)
{
    /* periodic boundaries; coordinates already inside skip the divisions */
    if (x < 0 || x >= L)
        x = ((x % L) + L) % L;
    if (y < 0 || y >= L)
        y = ((y % L) + L) % L;
    return s[y * L + x];
}

struct sweep_tables {
    uint32_t T4, T8;                  /* Ising: e^{-4 beta}, e^{-8 beta} */
    uint64_t lut[16];                 /* Ising with table-driven random bits */
    uint32_t thr[3][2][9];            /* Blume-Capel: [s+1][b][h+4] */
    int      always[3][2][9];
};

static void build_tables(struct sweep_tables* tb, int model, double beta, double D)
{
    int si, b, hi;
    memset(tb, 0, sizeof(*tb));
    if (model == ORA_ISING_LUT) {
        ora_lut_table(beta, tb->lut);
        return;
    }
    if (model == ORA_ISING) {
        tb->T4 = ora_threshold(beta, 4.0);
        tb->T8 = ora_threshold(beta, 8.0);
        return;
    }
    for (si = 0; si < 3; si++)
        for (b = 0; b < 2; b++)
            for (hi = 0; hi < 9; hi++) {
                int s = si - 1, h = hi - 4;
                int s2 = bc_propose(s, b);
                double dE = bc_delta_e(s, s2, h, D);
                if (dE <= 0.0) {
                    tb->always[si][b][hi] = 1;
                    tb->thr[si][b][hi] = 0;
                } else {
                    tb->always[si][b][hi] = 0;
                    tb->thr[si][b][hi] = ora_threshold(beta, dE);
                }
            }
}

/* One site update; returns the bond-sum change and sets *dq. */
static int64_t update_site(int8_t* s, int model, int64_t L, uint64_t seed, uint32_t t,
                           int color, int64_t x, int64_t y,
                           const struct sweep_tables* tb, int64_t* dq)
{
    int64_t n = y * L + x;
    uint64_t k = (uint64_t)n >> 1;
    int sv = s[n];
    int nb[4];
    int h;
    nb[0] = at(s, L, x + 1, y);
    nb[1] = at(s, L, x - 1, y);
    nb[2] = at(s, L, x, y + 1);
    nb[3] = at(s, L, x, y - 1);
    h = nb[0] + nb[1] + nb[2] + nb[3];
    *dq = 0;

    if (model == ORA_ISING_LUT) {
        /* section 3.2: a spin with at most two aligned neighbours flips; with
         * three it flips when its stream-0 bit (probability p = e^{-4 beta}) is
         * set; with four when both its stream-0 and stream-1 bits are set
         * (probability p^2 = e^{-8 beta}). */
        int aligned = (nb[0] == sv) + (nb[1] == sv) + (nb[2] == sv) + (nb[3] == sv);
        int flip;
        if (aligned <= 2) {
            flip = 1;
        } else {
            uint64_t g = k >> 2;
            int j = (int)(k & 3);
            int exp4 = (ora_lut_lookup(tb->lut, ora_lut_draw(seed, t, color, 0, g)) >> j) & 1;
            if (aligned == 3) {
                flip = exp4;
            } else {
                int exp8 = (ora_lut_lookup(tb->lut, ora_lut_draw(seed, t, color, 1, g)) >> j) & 1;
                flip = exp8 & exp4;
            }
        }
        if (flip) {
            s[n] = (int8_t)(-sv);
            return (int64_t)(-2 * sv * h);
        }
        return 0;
    }
    if (model == ORA_ISING) {
        int aligned = (nb[0] == sv) + (nb[1] == sv) + (nb[2] == sv) + (nb[3] == sv);
        int flip;
        if (aligned <= 2) {
            flip = 1;
        } else {
            uint32_t u = ora_accept_draw(seed, t, color, k);
            flip = (u < (aligned == 3 ? tb->T4 : tb->T8));
        }
        if (flip) {
            s[n] = (int8_t)(-sv);
            return (int64_t)(-2 * sv * h);
        }
        return 0;
    } else {
        int b = ora_proposal_bit(seed, t, color, k);
        int s2 = bc_propose(sv, b);
        int accept;
        if (tb->always[sv + 1][b][h + 4]) {
            accept = 1;
        } else {
            uint32_t u = ora_accept_draw(seed, t, color, k);
            accept = (u < tb->thr[sv + 1][b][h + 4]);
        }
        if (accept) {
            s[n] = (int8_t)s2;
            *dq = (int64_t)(s2 * s2 - sv * sv);
            return (int64_t)((s2 - sv) * h);
        }
        return 0;
    }
}

int ora_sweep(int8_t* s, int model, int64_t L, uint64_t seed, int64_t t0,
              int64_t n, double beta, double D, int nthreads,
              int64_t* dB, int64_t* dQ)
{
    struct sweep_tables tb;
    int64_t it;
    int64_t accB = 0, accQ = 0;
    if (L < 3) return -1;
    if (model != ORA_ISING && model != ORA_BC && model != ORA_ISING_LUT) return -1;
    if (beta != beta || beta < 0.0) return -2;
    if (D != D) return -3;
    if (t0 < 0 || n < 0 || t0 + n > 4294967296LL) return -4;
    build_tables(&tb, model, beta, D);

    for (it = 0; it < n; it++) {
        uint32_t t = (uint32_t)(t0 + it);
        int color;
        for (color = 0; color < 2; color++) {
            int64_t y;
            if (nthreads > 1 && (L % 2) == 0) {
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) reduction(+ : accB, accQ) schedule(static)
#endif
                for (y = 0; y < L; y++) {
                    int64_t x;
                    for (x = ((y + color) & 1); x < L; x += 2) {
                        int64_t dq;
                        accB += update_site(s, model, L, seed, t, color, x, y, &tb, &dq);
                        accQ += dq;
                    }
                }
            } else {
                for (y = 0; y < L; y++) {
                    int64_t x;
                    for (x = 0; x < L; x++) {
                        int64_t dq;
                        if (((x + y) & 1) != color) continue;
                        accB += update_site(s, model, L, seed, t, color, x, y, &tb, &dq);
                        accQ += dq;
                    }
                }
            }
        }
    }
    if (dB) *dB += accB;
    if (dQ) *dQ += accQ;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Measurements.  The paper names energy-like sums (section 4) and a spin    */
/* count check (Table 3 caption); reading: integer sums B (bond sum, so      */
/* E = -B + D Q), M, Q and the number of spins of each value.                */
/* ------------------------------------------------------------------------ */
void ora_measure(const int8_t* s, int64_t L, int64_t* B, int64_t* M, int64_t* Q,
                 int64_t counts[3], int nthreads)
{
    int64_t y, b = 0, m = 0, q = 0, c0 = 0, c1 = 0, c2 = 0;
    if (nthreads < 1) nthreads = 1;
    /* plain sums; with nthreads > 1 the rows are split over OpenMP threads
     * (integer sums, so the result does not depend on the split) */
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) reduction(+ : b, m, q, c0, c1, c2) schedule(static)
#endif
    for (y = 0; y < L; y++) {
        int64_t x;
        for (x = 0; x < L; x++) {
            int v = s[y * L + x];
            b += v * (at(s, L, x + 1, y) + at(s, L, x, y + 1));
            m += v;
            q += v * v;
            if (v == -1) c0++;
            else if (v == 0) c1++;
            else if (v == 1) c2++;
        }
    }
    *B = b; *M = m; *Q = q;
    counts[0] = c0; counts[1] = c1; counts[2] = c2;
}

/* ------------------------------------------------------------------------ */
/* Correlation protocol (section 3.3).  R = 16.  All sources for r <= 2R;    */
/* one source per R x R square (reading: the corner x = y = 0 mod R) for     */
/* 2R < r <= r_c(t); the same sampled sources on the log-spaced distances    */
/* floor(2^{x/32}) beyond r_c(t), up to L/2.                                 */
/*   r_c(t) = max{256, floor(g(L) sqrt(t) + 0.5)},                           */
/*   g(L)   = 6 sqrt(log(L / 2^16) / 3.3^2 + 1)  (reading: natural log),     */
/*   the log-spaced set keeps floor(2^{x/32}) > r_c(t), 1 <= x <= 32 log2(L/2)*/
/*   (reading of the printed condition, which compares x with r_c).          */
/* FULL mode: every distance 0..L/2, every source.                           */
/* ------------------------------------------------------------------------ */
#define CORR_R 16

double ora_g(int64_t L)
{
    return 6.0 * sqrt(log((double)L / 65536.0) / (3.3 * 3.3) + 1.0);
}

int64_t ora_rc(int64_t L, int64_t t)
{
    int64_t v = (int64_t)floor(ora_g(L) * sqrt((double)t) + 0.5);
    return v > 256 ? v : 256;
}

/* The three parts of the set are increasing and lie in disjoint ranges
 * (<= 2R, then (2R, r_c], then > r_c), so a repeat can only be the value
 * just appended (two log-spaced exponents can floor to the same distance). */
static int push_unique(int32_t* r, int cap, int count, int32_t v)
{
    if (count > 0 && count <= cap && r[count - 1] == v) return count;
    if (count < cap) r[count] = v;
    return count + 1;
}

int ora_rset(int mode, int64_t L, int64_t t, int32_t* r, int cap)
{
    int count = 0;
    int64_t half = L / 2, v;
    if (mode == ORA_CORR_FULL) {
        for (v = 0; v <= half; v++) count = push_unique(r, cap, count, (int32_t)v);
    } else {
        int64_t rc = ora_rc(L, t);
        int64_t x, xmax;
        for (v = 0; v <= half && v <= 2 * CORR_R; v++)
            count = push_unique(r, cap, count, (int32_t)v);
        for (v = 2 * CORR_R + 1; v <= half && v <= rc; v++)
            count = push_unique(r, cap, count, (int32_t)v);
        xmax = (int64_t)floor(32.0 * log2((double)L / 2.0) + 1e-9);
        for (x = 1; x <= xmax; x++) {
            int64_t d = (int64_t)floor(pow(2.0, (double)x / 32.0));
            if (d > rc && d <= half) count = push_unique(r, cap, count, (int32_t)d);
        }
    }
    if (count > cap) return -count;
    return count;
}

void ora_corr(const int8_t* s, int64_t L, int mode, const int32_t* r, int nr,
              int64_t* Cx, int64_t* Cy, int64_t* nsrc, int nthreads)
{
    int j;
    if (nthreads < 1) nthreads = 1;
    for (j = 0; j < nr; j++) {
        int64_t d = r[j], y, sx = 0, sy = 0, cnt = 0;
        int sampled = (mode == ORA_CORR_PROTOCOL) && d > 2 * CORR_R;
        /* rows split over OpenMP threads when nthreads > 1 (integer sums) */
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) reduction(+ : sx, sy, cnt) schedule(static)
#endif
        for (y = 0; y < L; y++) {
            int64_t x;
            if (sampled && (y % CORR_R) != 0) continue;         /* source rows y = 0 (mod R) */
            for (x = 0; x < L; x++) {
                int v;
                if (sampled && (x % CORR_R) != 0) continue;     /* source columns x = 0 (mod R) */
                v = s[y * L + x];
                sx += v * at(s, L, x + d, y);
                sy += v * at(s, L, x, y + d);
                cnt++;
            }
        }
        Cx[j] = sx; Cy[j] = sy; nsrc[j] = cnt;
    }
}

/* Schwinger-Dyson identity (eq. SDI): the sum of exp(-2 beta sigma h) takes
 * as many distinct values as sigma*h does, so a histogram of sigma*h over
 * the lattice is all a device needs to count. */
void ora_sd_hist(const int8_t* s, int64_t L, int64_t hist[9], int nthreads)
{
    int64_t y, h0 = 0, h1 = 0, h2 = 0, h3 = 0, h4 = 0, h5 = 0, h6 = 0, h7 = 0, h8 = 0;
    if (nthreads < 1) nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) reduction(+ : h0, h1, h2, h3, h4, h5, h6, h7, h8) schedule(static)
#endif
    for (y = 0; y < L; y++) {
        int64_t x;
        int64_t row[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (x = 0; x < L; x++) {
            int v = s[y * L + x];
            int h = at(s, L, x + 1, y) + at(s, L, x - 1, y) + at(s, L, x, y + 1) + at(s, L, x, y - 1);
            row[v * h + 4]++;
        }
        h0 += row[0]; h1 += row[1]; h2 += row[2]; h3 += row[3]; h4 += row[4];
        h5 += row[5]; h6 += row[6]; h7 += row[7]; h8 += row[8];
    }
    hist[0] = h0; hist[1] = h1; hist[2] = h2; hist[3] = h3; hist[4] = h4;
    hist[5] = h5; hist[6] = h6; hist[7] = h7; hist[8] = h8;
}

int ora_series(int8_t* s, int model, int64_t L, uint64_t seed, int64_t t0, int64_t n,
               double beta, double D, int64_t* Bs, int64_t* Ms, int64_t* Qs)
{
    int64_t i, cnt[3];
    for (i = 0; i < n; i++) {
        int rc = ora_sweep(s, model, L, seed, t0 + i, 1, beta, D, 1, NULL, NULL);
        if (rc) return rc;
        ora_measure(s, L, &Bs[i], &Ms[i], &Qs[i], cnt, 1);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Light-cone windows (see oracle.h).  The rule is the one of update_site,  */
/* evaluated at global coordinates; only the bookkeeping of which sites are */
/* present differs.                                                         */
/* ------------------------------------------------------------------------ */
static int init_value(int model, uint64_t seed, int init_state, uint64_t n)
{
    if (init_state == ORA_INIT_UP) return 1;
    if (init_state == ORA_INIT_DOWN) return -1;
    if (init_state == ORA_INIT_ZERO) return 0;
    {
        uint32_t w = ora_init_draw(seed, n);
        if (model != ORA_BC) return (w < 0x80000000u) ? 1 : -1;
        return (int)(((uint64_t)w * 3u) >> 32) - 1;
    }
}

int ora_init_window(int8_t* patch, int64_t P, int64_t x0, int64_t y0, int model, int64_t L, uint64_t seed,
                    int init_state)
{
    int64_t i, j;
    if (L < 3 || P < 3 || P > L) return -1;
    if (model != ORA_ISING && model != ORA_BC && model != ORA_ISING_LUT) return -1;
    if (init_state == ORA_INIT_ZERO && model != ORA_BC) return -1;
    for (j = 0; j < P; j++)
        for (i = 0; i < P; i++) {
            int64_t x = ((x0 + i) % L + L) % L, y = ((y0 + j) % L + L) % L;
            patch[j * P + i] = (int8_t)init_value(model, seed, init_state, (uint64_t)(y * L + x));
        }
    return 0;
}

int ora_sweep_window(int8_t* patch, int64_t P, int64_t x0, int64_t y0, int model, int64_t L, uint64_t seed,
                     int64_t t0, int64_t n, double beta, double D)
{
    struct sweep_tables tb;
    int64_t it;
    if (L < 3 || P < 3 || P > L || (L % 2) != 0) return -1;
    if (model != ORA_ISING && model != ORA_BC && model != ORA_ISING_LUT) return -1;
    if (beta != beta || beta < 0.0) return -2;
    if (D != D) return -3;
    if (t0 < 0 || n < 0 || t0 + n > 4294967296LL) return -4;
    build_tables(&tb, model, beta, D);
    for (it = 0; it < n; it++) {
        uint32_t t = (uint32_t)(t0 + it);
        int color;
        for (color = 0; color < 2; color++) {
            int64_t i, j;
            for (j = 1; j < P - 1; j++)
                for (i = 1; i < P - 1; i++) {
                    int64_t x = ((x0 + i) % L + L) % L, y = ((y0 + j) % L + L) % L;
                    int8_t* c = &patch[j * P + i];
                    int sv = *c, nb[4], h, s2;
                    uint64_t k;
                    if (((x + y) & 1) != color) continue;
                    k = (uint64_t)(y * L + x) >> 1;
                    nb[0] = patch[j * P + i + 1];
                    nb[1] = patch[j * P + i - 1];
                    nb[2] = patch[(j + 1) * P + i];
                    nb[3] = patch[(j - 1) * P + i];
                    h = nb[0] + nb[1] + nb[2] + nb[3];
                    if (model == ORA_ISING) {
                        int aligned = (nb[0] == sv) + (nb[1] == sv) + (nb[2] == sv) + (nb[3] == sv);
                        int flip = aligned <= 2;
                        if (!flip) flip = ora_accept_draw(seed, t, color, k) < (aligned == 3 ? tb.T4 : tb.T8);
                        if (flip) *c = (int8_t)(-sv);
                    } else if (model == ORA_ISING_LUT) {
                        int aligned = (nb[0] == sv) + (nb[1] == sv) + (nb[2] == sv) + (nb[3] == sv);
                        int flip = aligned <= 2;
                        if (!flip) {
                            int j = (int)(k & 3);
                            int e4 = (ora_lut_lookup(tb.lut, ora_lut_draw(seed, t, color, 0, k >> 2)) >> j) & 1;
                            flip = e4;
                            if (aligned == 4 && e4)
                                flip = (ora_lut_lookup(tb.lut, ora_lut_draw(seed, t, color, 1, k >> 2)) >> j) & 1;
                        }
                        if (flip) *c = (int8_t)(-sv);
                    } else {
                        int b = ora_proposal_bit(seed, t, color, k);
                        int accept = tb.always[sv + 1][b][h + 4];
                        s2 = bc_propose(sv, b);
                        if (!accept) accept = ora_accept_draw(seed, t, color, k) < tb.thr[sv + 1][b][h + 4];
                        if (accept) *c = (int8_t)s2;
                    }
                }
        }
    }
    return 0;
}
