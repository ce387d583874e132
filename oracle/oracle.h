/*
 * CPU oracle for the checkerboard Metropolis sweep of the 2D Ising and
 * Blume-Capel models and for the measurements taken during the relaxation
 * after a quench (Bisson et al., "Massive-Scale Simulations of 2D Ising and
 * Blume-Capel Models on Rack-Scale Multi-GPU Systems", arXiv:2502.18624).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (the HIP library and its Python binding) never links, imports or calls it.
 * It shares no code, header, table or constant generator with the product.
 *
 * Plain, slow, obviously correct: an int8 array s[y*L + x] with x the fast
 * axis, periodic boundaries, scalar loops, fp64 on the host for the
 * acceptance thresholds.  Each function cites the passage of the paper that
 * defines what it computes; where the paper is silent the reading taken is
 * stated next to the function (and listed with the other readings in the
 * design notes of the repository).
 */
#ifndef ORACLE_H
#define ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_ISING = 0, ORA_BC = 1, ORA_ISING_LUT = 2 };
enum { ORA_INIT_RANDOM = 0, ORA_INIT_UP = 1, ORA_INIT_DOWN = 2, ORA_INIT_ZERO = 3 };
enum { ORA_CORR_FULL = 1, ORA_CORR_PROTOCOL = 2 };

/* Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11); the
 * paper draws its uniforms from this generator (section 3.2). */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The three random streams of the counter contract (reading of the paper's
 * unstated RNG layout; all keyed by the logical site, never by storage). */
uint32_t ora_accept_draw(uint64_t seed, uint32_t t, int color, uint64_t k);
int      ora_proposal_bit(uint64_t seed, uint32_t t, int color, uint64_t k);
uint32_t ora_init_draw(uint64_t seed, uint64_t n);

/* Non-uniform random bits of section 3.2 (model ORA_ISING_LUT): 16 sorted
 * thresholds T[k] = floor(2^32 C_k), C_k the probability of the 4-bit
 * patterns 0..k-1 when each bit is set independently with p = exp(-4 beta);
 * a 32-bit uniform u selects the pattern max{k : T[k] <= u}.  T[k] may be
 * 2^32 (never selected), hence 64-bit. */
void     ora_lut_table(double beta, uint64_t T[16]);
int      ora_lut_lookup(const uint64_t T[16], uint32_t u);
/* The draw feeding the 4 random bits of in-colour sites 4g .. 4g+3, for
 * stream e (0: exp4, 1: the word ANDed into exp8). */
uint32_t ora_lut_draw(uint64_t seed, uint32_t t, int color, int e, uint64_t g);

/* Acceptance threshold floor(2^32 exp(-beta dE)) clamped to 2^32-1, dE > 0. */
uint32_t ora_threshold(double beta, double dE);

/* Probability with which the oracle's update rule accepts a move; for the
 * Ising model `aligned` is the number of neighbours equal to the spin (the
 * section 3.2 rule), for Blume-Capel (s, h, b) give the proposal. */
double ora_ising_flip_prob(int aligned, double beta);
double ora_bc_accept_prob(int s, int h, int b, double beta, double D);

int  ora_init(int8_t* s, int model, int64_t L, uint64_t seed, int init_state);

/* n sweeps starting at sweep index t0.  If dB/dQ are non-NULL they
 * accumulate the bond-sum and sum-of-squares changes of every accepted move.
 * nthreads > 1 splits the rows of one colour over OpenMP threads (even L). */
int  ora_sweep(int8_t* s, int model, int64_t L, uint64_t seed, int64_t t0,
               int64_t n, double beta, double D, int nthreads,
               int64_t* dB, int64_t* dQ);

/* B = sum s(x,y)[s(x+1,y)+s(x,y+1)], M = sum s, Q = sum s^2, counts of -1,0,+1.
 * nthreads > 1 splits the rows over OpenMP threads (same integer sums). */
void ora_measure(const int8_t* s, int64_t L, int64_t* B, int64_t* M, int64_t* Q,
                 int64_t counts[3], int nthreads);

/* Distances of the correlation function (section 3.3).  Returns the number
 * of distances, or -(needed) if cap is too small. */
int  ora_rset(int mode, int64_t L, int64_t t, int32_t* r, int cap);
int64_t ora_rc(int64_t L, int64_t t);
double  ora_g(int64_t L);

/* S_a(r) = sum over sources p of s(p) s(p + r e_a), a in {x, y}; nthreads as
 * for ora_measure. */
void ora_corr(const int8_t* s, int64_t L, int mode, const int32_t* r, int nr,
              int64_t* Cx, int64_t* Cy, int64_t* nsrc, int nthreads);

/* Schwinger-Dyson histogram: hist[k] = #sites with sigma*h = k - 4. */
void ora_sd_hist(const int8_t* s, int64_t L, int64_t hist[9], int nthreads);

/* Light-cone windows of a large lattice.  patch[P*P] holds the sites
 * (x0 + i, y0 + j) mod L of an L x L lattice (row j, column i).  The
 * window init writes their initial state; the window sweep applies the same
 * update rule with colours and random draws of the global coordinates, to
 * the sites whose four neighbours lie in the patch (the outer ring stays
 * frozen).  After n sweeps the sites at least 2n from the patch edge equal
 * those of the full lattice: a half-sweep moves information by one site. */
int ora_init_window(int8_t* patch, int64_t P, int64_t x0, int64_t y0, int model, int64_t L, uint64_t seed,
                    int init_state);
int ora_sweep_window(int8_t* patch, int64_t P, int64_t x0, int64_t y0, int model, int64_t L, uint64_t seed,
                     int64_t t0, int64_t n, double beta, double D);

/* Runs n sweeps one at a time and records B, M, Q after each. */
int  ora_series(int8_t* s, int model, int64_t L, uint64_t seed, int64_t t0, int64_t n,
                double beta, double D, int64_t* Bs, int64_t* Ms, int64_t* Qs);

#ifdef __cplusplus
}
#endif
#endif
