/*
 * fc_oracle.h -- plain FP64 CPU oracle of the Feldman-Cousins grid scan.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two meet only through the
 * seeded input generator.
 *
 * What it computes (arXiv:2002.07858):
 *   - Eq. (1) / Algorithm 2: chi^2 = (a-b)^T M (a-b), with M the inverse of an
 *     SPD covariance.  Evaluated here as ||L^{-1}(a-b)||^2 by forward
 *     substitution with the Cholesky factor L of the covariance, so no
 *     inverse is ever formed.
 *   - Section 2 (grid): the D-dimensional rectangular grid is linearised into
 *     a list, row-major with the last axis fastest.
 *   - Algorithm 1: per universe, strict "<" running minimum over the grid in
 *     list order, initialised to +inf with the minimiser set to the true
 *     point; Delta chi^2 = chi^2 at the true point minus the minimum.
 *   - Section 1 / Figure 1: critical values are the values left of which a
 *     stated fraction of the Delta chi^2 distribution lies (type-1 order
 *     statistic), plus a fixed-bin histogram.
 * The covariance at grid point q is Sigma_q = diag(stat) + F o (S_q S_q^T):
 * Pearson statistical term stat = S_q (or a fixed stat vector) plus a
 * fractional systematic matrix F scaled by the prediction.
 *
 * All arithmetic is IEEE FP64, compiled without FP contraction.
 */
#ifndef FC_ORACLE_H
#define FC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCO_STAT_PEARSON 0
#define FCO_STAT_FIXED 1

/* Coordinates of linear grid index q: coords[d] = axis_vals[off_d + i_d]. */
int fco_grid_coords(int32_t D, const int64_t *axis_len, const double *axis_vals,
                    int64_t q, double *coords);

/* Sigma = diag(stat) + F o (s s^T), row-major [N][N]. */
int fco_covariance(int32_t N, const double *s, const double *F, int32_t stat_mode,
                   const double *stat_diag, double *Sigma);

/* Lower Cholesky factor of A ([N][N] row-major) into L ([N][N], upper part
 * zeroed).  Returns 0, or -1 if a pivot is not > 0 (not positive definite). */
int fco_cholesky(int32_t N, const double *A, double *L);

/* chi^2 = ||L^{-1}(a-b)||^2 by forward substitution, L full [N][N]. */
double fco_chi2(int32_t N, const double *L, const double *a, const double *b);

/* Cholesky factors of Sigma_q for q = q0 .. q0+nq-1, written as full
 * [nq][N][N] (S is the whole [G][N] table).  On failure returns -2 and sets
 * *bad_q to the first q that is not PD, else *bad_q = -1. */
int fco_factor_range(int64_t G, int32_t N, const double *S, const double *F,
                     int32_t stat_mode, const double *stat_diag, int64_t q0, int64_t nq,
                     double *L_blk, int64_t *bad_q, int32_t nthreads);

/* Algorithm 1 for K universes d[K][N] with true points p_idx[K].
 * Outputs per universe: dchi2, chi2_min, argmin, chi2_p (chi^2 at the true
 * point) and chi2_2nd (smallest chi^2 at a grid point other than argmin,
 * +inf if G == 1).  Returns -1 on a bad argument. */
int fco_scan(int64_t G, int32_t N, const double *S, const double *L_all, int64_t K,
             const double *d, const int64_t *p_idx, double *dchi2, double *chi2_min,
             int64_t *argmin, double *chi2_p, double *chi2_2nd, int32_t nthreads);

/* The same scan split in three so that very large grids can be walked in
 * consecutive ranges of q without holding every factor at once:
 *   init   : chi2_min = +inf, argmin = p, chi2_p = NaN, chi2_2nd = +inf
 *   range  : continue every universe's running minimum over q0 .. q0+nq-1 in
 *            order, with L_blk holding the factors of those nq points
 *   finish : dchi2 = chi2_p - chi2_min
 * Calling range over 0..G-1 in increasing, contiguous pieces gives exactly the
 * result of one pass over the whole grid. */
int fco_scan_init(int64_t K, const int64_t *p_idx, double *chi2_min, int64_t *argmin,
                  double *chi2_p, double *chi2_2nd);
int fco_scan_range(int64_t G, int32_t N, const double *S, int64_t q0, int64_t nq,
                   const double *L_blk, int64_t K, const double *d, const int64_t *p_idx,
                   double *chi2_min, int64_t *argmin, double *chi2_p, double *chi2_2nd,
                   int32_t nthreads);
int fco_scan_finish(int64_t K, const double *chi2_p, const double *chi2_min, double *dchi2);

/* chi^2 of every universe against every grid point: out[K][G]. */
int fco_chi2_table(int64_t G, int32_t N, const double *S, const double *L_all, int64_t K,
                   const double *d, double *out, int32_t nthreads);

/* Per segment s (values x[seg_off[s] .. seg_off[s+1])): crit[s][a] is the
 * j-th smallest value, j = ceil(alpha[a] * K_s) clamped to [1, K_s] (NaN sorts
 * last; NaN for an empty segment); hist[s][b], b < n_bins, counts values with
 * 0 <= x < hist_hi in bin floor(x / (hist_hi / n_bins)) (clamped to n_bins-1);
 * hist[s][n_bins] counts everything else, NaN included.  hist may be NULL. */
int fco_critical_value(int64_t n_seg, const int64_t *seg_off, const double *x,
                       int32_t n_alpha, const double *alpha, double *crit,
                       int32_t n_bins, double hist_hi, int64_t *hist);

/* Algorithm 1 as printed, with one matrix M for the whole grid: per universe
 * M = Sigma_m^{-1} with m the true point; with max_iter > 0, step 5 of the
 * procedure in Section 2: after a scan, if the minimiser q_min differs from
 * m, set m = q_min and scan again (at most max_iter times).  chi2(d, q) =
 * (d - S_q)^T M (d - S_q) via the Cholesky factor of Sigma_m; Delta chi2 =
 * chi2(d, S_p) - min, both with the last M.  Outputs per universe: dchi2,
 * chi2_min, argmin, chi2_p, m_final, iters (re-scans done).  Returns -2 if a
 * covariance is not positive definite. */
int fco_scan_fixed_m(int64_t G, int32_t N, const double *S, const double *F, int32_t stat_mode,
                     const double *stat_diag, int64_t K, const double *d, const int64_t *p_idx,
                     int32_t max_iter, double *dchi2, double *chi2_min, int64_t *argmin,
                     double *chi2_p, int64_t *m_final, int32_t *iters, int32_t nthreads);

/* ---- universes (Section 2, steps 1-2: fluctuate the prediction at p) -----
 *
 * Counter-based stream, the same definition on every side:
 *   Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
 *     (hi0,lo0) = mulhilo(0xD2E7470EE14C6C93, x0), (hi1,lo1) = mulhilo(0xCA5A826395121157, x2),
 *     x = (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0),
 *   the key advancing by (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B) after each round.
 *   Key (seed, 0).  Block b of purpose t for true point p, universe j, bin i
 *   has counter (j, p, i << 32 | t << 28 | b, 0); t = 0 Poisson, t = 1 normal.
 *   A 64-bit word w gives the uniform ((w >> 11) + 0.5) * 2^-53 in (0, 1).
 * Poisson(lambda): lambda = 0 -> 0; lambda < 10: multiplication method (the
 *   product of uniforms, words in block order, first at or below
 *   exp(-lambda); at most 1024 uniforms); lambda >= 10: Hormann's transformed
 *   rejection with squeeze (PTRS, 1993), attempt t taking words 2(t%2),
 *   2(t%2)+1 of block t/2, at most 512 attempts, then floor(lambda).
 *   lambda < 0, NaN or inf -> -1 (no value).
 * Normal: sqrt(-2 ln u0) cos(2 pi u1) from words 0, 1 of the bin's normal block.
 * Universe: d_i = n_i + S_p[i] * sum_{l <= i} LF[i][l] g_l, LF = chol(F),
 *   summed in increasing l (n_i = -1 gives d_i = NaN). */
void fco_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double fco_uniform(uint64_t w);
int64_t fco_poisson(double lambda, uint64_t seed, int64_t p, int64_t j, int32_t i);
double fco_normal(uint64_t seed, int64_t p, int64_t j, int32_t i);
/* Universes of n_pts true points: rows seg_off[k] .. seg_off[k+1]-1 are
 * universes u_first[k] + 0, 1, ... of point p[k] (u_first may be NULL = 0).
 * LF is chol(F) [N][N].  counts may be NULL.  Returns -1 on a bad argument. */
int fco_universes(int64_t G, int32_t N, const double *S, const double *LF, int64_t n_pts,
                  const int64_t *p, const int64_t *seg_off, const int64_t *u_first,
                  uint64_t seed, double *d, int32_t *counts, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
