/*
 * fc_oracle.c -- plain FP64 CPU oracle of the Feldman-Cousins grid scan.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library, with which it
 * shares no code.  See fc_oracle.h for what each function computes and which
 * part of arXiv:2002.07858 it follows.
 *
 * The code is deliberately plain: textbook Cholesky, forward substitution,
 * loops in the order the paper states them.  Threads only split the
 * independent universes (Algorithm 1's outer loop) or grid points (the
 * covariance factors) into static contiguous ranges.
 */
#include "fc_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ---- Section 2: grid linearisation (last axis fastest) ------------------ */
int fco_grid_coords(int32_t D, const int64_t *axis_len, const double *axis_vals,
                    int64_t q, double *coords)
{
    if (D <= 0 || !axis_len || !axis_vals || !coords || q < 0) return -1;
    int64_t G = 1;
    for (int32_t e = 0; e < D; ++e) {
        if (axis_len[e] <= 0) return -1;
        G *= axis_len[e];
    }
    if (q >= G) return -1;
    /* q = sum_d i_d * prod_{e>d} n_e : peel indices from the last axis. */
    int64_t off[64];
    if (D > 64) return -1;
    int64_t o = 0;
    for (int32_t e = 0; e < D; ++e) { off[e] = o; o += axis_len[e]; }
    int64_t rest = q;
    for (int32_t e = D - 1; e >= 0; --e) {
        int64_t i = rest % axis_len[e];
        rest /= axis_len[e];
        coords[e] = axis_vals[off[e] + i];
    }
    return 0;
}

/* ---- covariance: statistical diagonal + fractional systematic ------------ */
int fco_covariance(int32_t N, const double *s, const double *F, int32_t stat_mode,
                   const double *stat_diag, double *Sigma)
{
    if (N <= 0 || !s || !F || !Sigma) return -1;
    if (stat_mode == FCO_STAT_FIXED && !stat_diag) return -1;
    if (stat_mode != FCO_STAT_PEARSON && stat_mode != FCO_STAT_FIXED) return -1;
    for (int32_t i = 0; i < N; ++i) {
        for (int32_t j = 0; j < N; ++j) {
            double v = F[(int64_t)i * N + j] * (s[i] * s[j]);
            if (i == j) v += (stat_mode == FCO_STAT_PEARSON) ? s[i] : stat_diag[i];
            Sigma[(int64_t)i * N + j] = v;
        }
    }
    return 0;
}

/* ---- textbook Cholesky-Banachiewicz, row by row ------------------------- */
int fco_cholesky(int32_t N, const double *A, double *L)
{
    for (int64_t t = 0; t < (int64_t)N * N; ++t) L[t] = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        for (int32_t j = 0; j <= i; ++j) {
            double sum = A[(int64_t)i * N + j];
            for (int32_t k = 0; k < j; ++k)
                sum -= L[(int64_t)i * N + k] * L[(int64_t)j * N + k];
            if (i == j) {
                if (!(sum > 0.0)) return -1; /* not positive definite (or NaN) */
                L[(int64_t)i * N + i] = sqrt(sum);
            } else {
                L[(int64_t)i * N + j] = sum / L[(int64_t)j * N + j];
            }
        }
    }
    return 0;
}

/* ---- Eq. (1): chi^2 = r^T Sigma^{-1} r = ||y||^2 with L y = r ------------- */
double fco_chi2(int32_t N, const double *L, const double *a, const double *b)
{
    double y[256];
    double chi2 = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        double v = a[i] - b[i];
        for (int32_t k = 0; k < i; ++k) v -= L[(int64_t)i * N + k] * y[k];
        y[i] = v / L[(int64_t)i * N + i];
        chi2 += y[i] * y[i];
    }
    return chi2;
}

/* ---- static thread ranges -------------------------------------------------- */
typedef void (*fco_task_fn)(void *ctx, int64_t lo, int64_t hi);

struct fco_task {
    fco_task_fn fn;
    void *ctx;
    int64_t lo, hi;
};

static void *fco_task_run(void *arg)
{
    struct fco_task *t = (struct fco_task *)arg;
    t->fn(t->ctx, t->lo, t->hi);
    return NULL;
}

static void fco_parallel(int64_t n, int32_t nthreads, fco_task_fn fn, void *ctx)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > n) nthreads = (int32_t)(n > 0 ? n : 1);
    if (nthreads == 1) { fn(ctx, 0, n); return; }
    pthread_t th[256];
    struct fco_task task[256];
    int started[256];
    for (int32_t t = 0; t < nthreads; ++t) {
        task[t].fn = fn;
        task[t].ctx = ctx;
        task[t].lo = n * t / nthreads;
        task[t].hi = n * (t + 1) / nthreads;
        started[t] = pthread_create(&th[t], NULL, fco_task_run, &task[t]) == 0;
        if (!started[t]) fn(ctx, task[t].lo, task[t].hi);
    }
    for (int32_t t = 0; t < nthreads; ++t)
        if (started[t]) pthread_join(th[t], NULL);
}

/* ---- factors of every Sigma_q in a range --------------------------------- */
struct fco_factor_ctx {
    int32_t N;
    const double *S, *F, *stat_diag;
    int32_t stat_mode;
    int64_t q0;
    double *L_blk;
    int64_t *first_bad; /* per thread-range result, merged afterwards */
    pthread_mutex_t mu;
};

static void fco_factor_task(void *vctx, int64_t lo, int64_t hi)
{
    struct fco_factor_ctx *c = (struct fco_factor_ctx *)vctx;
    int32_t N = c->N;
    double *Sigma = (double *)malloc(sizeof(double) * (size_t)N * (size_t)N);
    if (!Sigma) return;
    for (int64_t t = lo; t < hi; ++t) {
        int64_t q = c->q0 + t;
        fco_covariance(N, c->S + q * N, c->F, c->stat_mode, c->stat_diag, Sigma);
        if (fco_cholesky(N, Sigma, c->L_blk + t * (int64_t)N * N) != 0) {
            pthread_mutex_lock(&c->mu);
            if (*c->first_bad < 0 || q < *c->first_bad) *c->first_bad = q;
            pthread_mutex_unlock(&c->mu);
        }
    }
    free(Sigma);
}

int fco_factor_range(int64_t G, int32_t N, const double *S, const double *F,
                     int32_t stat_mode, const double *stat_diag, int64_t q0, int64_t nq,
                     double *L_blk, int64_t *bad_q, int32_t nthreads)
{
    if (G <= 0 || N <= 0 || N > 256 || !S || !F || !L_blk || !bad_q) return -1;
    if (q0 < 0 || nq < 0 || q0 + nq > G) return -1;
    if (stat_mode == FCO_STAT_FIXED && !stat_diag) return -1;
    struct fco_factor_ctx c;
    c.N = N; c.S = S; c.F = F; c.stat_diag = stat_diag; c.stat_mode = stat_mode;
    c.q0 = q0; c.L_blk = L_blk;
    int64_t first_bad = -1;
    c.first_bad = &first_bad;
    pthread_mutex_init(&c.mu, NULL);
    fco_parallel(nq, nthreads, fco_factor_task, &c);
    pthread_mutex_destroy(&c.mu);
    *bad_q = first_bad;
    return first_bad >= 0 ? -2 : 0;
}

/* ---- Algorithm 1 ---------------------------------------------------------- */
int fco_scan_init(int64_t K, const int64_t *p_idx, double *chi2_min, int64_t *argmin,
                  double *chi2_p, double *chi2_2nd)
{
    if (K < 0 || (K > 0 && (!p_idx || !chi2_min || !argmin || !chi2_p || !chi2_2nd))) return -1;
    for (int64_t k = 0; k < K; ++k) {
        chi2_min[k] = INFINITY; /* chi^2_min <- inf */
        argmin[k] = p_idx[k];   /* p_min = p        */
        chi2_p[k] = NAN;
        chi2_2nd[k] = INFINITY;
    }
    return 0;
}

struct fco_scan_ctx {
    int32_t N;
    const double *S, *L_blk, *d;
    const int64_t *p_idx;
    int64_t q0, nq;
    double *chi2_min, *chi2_p, *chi2_2nd;
    int64_t *argmin;
};

static void fco_scan_task(void *vctx, int64_t lo, int64_t hi)
{
    struct fco_scan_ctx *c = (struct fco_scan_ctx *)vctx;
    int32_t N = c->N;
    for (int64_t k = lo; k < hi; ++k) {           /* each universe ...        */
        const double *a = c->d + k * N;
        double best = c->chi2_min[k];
        double second = c->chi2_2nd[k];
        int64_t qbest = c->argmin[k];
        for (int64_t t = 0; t < c->nq; ++t) {     /* ... against every q, in order */
            int64_t q = c->q0 + t;
            double chi2 = fco_chi2(N, c->L_blk + t * (int64_t)N * N, a, c->S + q * N);
            if (q == c->p_idx[k]) c->chi2_p[k] = chi2;
            if (chi2 < best) {                    /* strict "<": first q wins ties */
                second = best;
                best = chi2;
                qbest = q;
            } else if (chi2 < second) {
                second = chi2;
            }
        }
        c->chi2_min[k] = best;
        c->chi2_2nd[k] = second;
        c->argmin[k] = qbest;
    }
}

int fco_scan_range(int64_t G, int32_t N, const double *S, int64_t q0, int64_t nq,
                   const double *L_blk, int64_t K, const double *d, const int64_t *p_idx,
                   double *chi2_min, int64_t *argmin, double *chi2_p, double *chi2_2nd,
                   int32_t nthreads)
{
    if (G <= 0 || N <= 0 || N > 256 || !S || q0 < 0 || nq < 0 || q0 + nq > G) return -1;
    if (K < 0 || (K > 0 && (!d || !p_idx || !chi2_min || !argmin || !chi2_p || !chi2_2nd)))
        return -1;
    if (nq > 0 && !L_blk) return -1;
    for (int64_t k = 0; k < K; ++k)
        if (p_idx[k] < 0 || p_idx[k] >= G) return -1;
    struct fco_scan_ctx c;
    c.N = N; c.S = S; c.L_blk = L_blk; c.d = d; c.p_idx = p_idx;
    c.q0 = q0; c.nq = nq;
    c.chi2_min = chi2_min; c.chi2_p = chi2_p; c.chi2_2nd = chi2_2nd; c.argmin = argmin;
    fco_parallel(K, nthreads, fco_scan_task, &c);
    return 0;
}

int fco_scan_finish(int64_t K, const double *chi2_p, const double *chi2_min, double *dchi2)
{
    if (K < 0 || (K > 0 && (!chi2_p || !chi2_min || !dchi2))) return -1;
    for (int64_t k = 0; k < K; ++k) dchi2[k] = chi2_p[k] - chi2_min[k];
    return 0;
}

int fco_scan(int64_t G, int32_t N, const double *S, const double *L_all, int64_t K,
             const double *d, const int64_t *p_idx, double *dchi2, double *chi2_min,
             int64_t *argmin, double *chi2_p, double *chi2_2nd, int32_t nthreads)
{
    int rc = fco_scan_init(K, p_idx, chi2_min, argmin, chi2_p, chi2_2nd);
    if (rc) return rc;
    rc = fco_scan_range(G, N, S, 0, G, L_all, K, d, p_idx, chi2_min, argmin, chi2_p,
                        chi2_2nd, nthreads);
    if (rc) return rc;
    return fco_scan_finish(K, chi2_p, chi2_min, dchi2);
}

/* ---- chi^2 of every (universe, grid point) pair ---------------------------- */
struct fco_table_ctx {
    int64_t G;
    int32_t N;
    const double *S, *L_all, *d;
    double *out;
};

static void fco_table_task(void *vctx, int64_t lo, int64_t hi)
{
    struct fco_table_ctx *c = (struct fco_table_ctx *)vctx;
    for (int64_t k = lo; k < hi; ++k)
        for (int64_t q = 0; q < c->G; ++q)
            c->out[k * c->G + q] = fco_chi2(c->N, c->L_all + q * (int64_t)c->N * c->N,
                                            c->d + k * c->N, c->S + q * c->N);
}

int fco_chi2_table(int64_t G, int32_t N, const double *S, const double *L_all, int64_t K,
                   const double *d, double *out, int32_t nthreads)
{
    if (G <= 0 || N <= 0 || N > 256 || !S || !L_all || K < 0 || (K > 0 && (!d || !out)))
        return -1;
    struct fco_table_ctx c = {G, N, S, L_all, d, out};
    fco_parallel(K, nthreads, fco_table_task, &c);
    return 0;
}

/* ---- critical values (type-1 order statistic) and histogram -------------- */
static int fco_cmp_nan_last(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    int an = isnan(a), bn = isnan(b);
    if (an || bn) return an - bn;
    return (a > b) - (a < b);
}

int fco_critical_value(int64_t n_seg, const int64_t *seg_off, const double *x,
                       int32_t n_alpha, const double *alpha, double *crit,
                       int32_t n_bins, double hist_hi, int64_t *hist)
{
    if (n_seg < 0 || !seg_off || n_alpha < 0 || (n_alpha > 0 && (!alpha || !crit))) return -1;
    if (hist && (n_bins <= 0 || !(hist_hi > 0.0))) return -1;
    for (int32_t a = 0; a < n_alpha; ++a)
        if (!(alpha[a] > 0.0 && alpha[a] <= 1.0)) return -1;
    for (int64_t s = 0; s < n_seg; ++s) {
        int64_t lo = seg_off[s], hi = seg_off[s + 1];
        if (lo < 0 || hi < lo) return -1;
        int64_t K = hi - lo;
        double *v = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
        if (!v) return -3;
        memcpy(v, x + lo, sizeof(double) * (size_t)K);
        qsort(v, (size_t)K, sizeof(double), fco_cmp_nan_last);
        for (int32_t a = 0; a < n_alpha; ++a) {
            if (K == 0) { crit[s * n_alpha + a] = NAN; continue; }
            double jr = ceil(alpha[a] * (double)K);
            int64_t j = (int64_t)jr;
            if (j < 1) j = 1;
            if (j > K) j = K;
            crit[s * n_alpha + a] = v[j - 1];
        }
        free(v);
        if (hist) {
            int64_t *h = hist + s * (int64_t)(n_bins + 1);
            for (int32_t b = 0; b <= n_bins; ++b) h[b] = 0;
            double width = hist_hi / (double)n_bins;
            for (int64_t k = lo; k < hi; ++k) {
                double xv = x[k];
                int64_t b = n_bins;
                if (xv >= 0.0 && xv < hist_hi) {
                    b = (int64_t)floor(xv / width);
                    if (b > n_bins - 1) b = n_bins - 1;
                }
                h[b] += 1;
            }
        }
    }
    return 0;
}

/* ---- universes: counter-based stream, Poisson and normal variates -------- */

/* 64 x 64 -> 128-bit product split into high and low words. */
static void fco_mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* Philox4x64 with 10 rounds (Salmon et al., SC'11). */
void fco_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        fco_mulhilo64(0xD2E7470EE14C6C93ull, x0, &hi0, &lo0);
        fco_mulhilo64(0xCA5A826395121157ull, x2, &hi1, &lo1);
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

double fco_uniform(uint64_t w)
{
    return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

static void fco_block(uint64_t seed, int64_t p, int64_t j, int32_t i, uint32_t purpose,
                      uint32_t b, uint64_t out[4])
{
    const uint64_t ctr[4] = {(uint64_t)j, (uint64_t)p,
                             ((uint64_t)(uint32_t)i << 32) | ((uint64_t)purpose << 28) | b, 0};
    const uint64_t key[2] = {seed, 0};
    fco_philox4x64(ctr, key, out);
}

int64_t fco_poisson(double lambda, uint64_t seed, int64_t p, int64_t j, int32_t i)
{
    if (!(lambda >= 0.0) || isinf(lambda)) return -1;
    if (lambda == 0.0) return 0;
    uint64_t w[4];
    if (lambda < 10.0) {
        /* multiplication method: count uniforms until their product first
         * falls to exp(-lambda) or below */
        const double L = exp(-lambda);
        double prod = 1.0;
        int64_t k = 0;
        for (uint32_t b = 0; b < 256; ++b) {
            fco_block(seed, p, j, i, 0, b, w);
            for (int e = 0; e < 4; ++e) {
                prod *= fco_uniform(w[e]);
                if (prod <= L) return k;
                ++k;
            }
        }
        return k;
    }
    /* PTRS: transformed rejection with squeeze (Hormann 1993) */
    const double slam = sqrt(lambda), loglam = log(lambda);
    const double bb = 0.931 + 2.53 * slam;
    const double aa = -0.059 + 0.02483 * bb;
    const double inv_alpha = 1.1239 + 1.1328 / (bb - 3.4);
    const double vr = 0.9277 - 3.6224 / (bb - 2.0);
    for (uint32_t t = 0; t < 512; ++t) {
        if ((t & 1) == 0) fco_block(seed, p, j, i, 0, t >> 1, w);
        const double U = fco_uniform(w[2 * (t & 1)]) - 0.5;
        const double V = fco_uniform(w[2 * (t & 1) + 1]);
        const double us = 0.5 - fabs(U);
        const double kf = floor((2.0 * aa / us + bb) * U + lambda + 0.43);
        if (us >= 0.07 && V <= vr) return (int64_t)kf;
        if (kf < 0.0 || (us < 0.013 && V > us)) continue;
        const double lhs = log(V * inv_alpha / (aa / (us * us) + bb));
        const double rhs = -lambda + kf * loglam - lgamma(kf + 1.0);
        if (lhs <= rhs) return (int64_t)kf;
    }
    return (int64_t)floor(lambda);
}

double fco_normal(uint64_t seed, int64_t p, int64_t j, int32_t i)
{
    uint64_t w[4];
    fco_block(seed, p, j, i, 1, 0, w);
    const double u0 = fco_uniform(w[0]), u1 = fco_uniform(w[1]);
    return sqrt(-2.0 * log(u0)) * cos(6.283185307179586 * u1);
}

struct fco_univ_ctx {
    int32_t N;
    const double *S, *LF;
    int64_t n_pts;
    const int64_t *p, *seg_off, *u_first;
    uint64_t seed;
    double *d;
    int32_t *counts;
};

static void fco_univ_task(void *vctx, int64_t lo, int64_t hi)
{
    struct fco_univ_ctx *c = (struct fco_univ_ctx *)vctx;
    const int32_t N = c->N;
    double g[64];
    for (int64_t k = lo; k < hi; ++k) {
        const int64_t p = c->p[k];
        const double *Sp = c->S + p * N;
        for (int64_t r = c->seg_off[k]; r < c->seg_off[k + 1]; ++r) {
            const int64_t j = (c->u_first ? c->u_first[k] : 0) + (r - c->seg_off[k]);
            for (int32_t i = 0; i < N; ++i) g[i] = fco_normal(c->seed, p, j, i);
            for (int32_t i = 0; i < N; ++i) {
                const int64_t n = fco_poisson(Sp[i], c->seed, p, j, i);
                double z = 0.0;
                for (int32_t l = 0; l <= i; ++l) z += c->LF[i * N + l] * g[l];
                c->d[r * N + i] = (n < 0) ? NAN : (double)n + Sp[i] * z;
                if (c->counts) c->counts[r * N + i] = (int32_t)n;
            }
        }
    }
}

int fco_universes(int64_t G, int32_t N, const double *S, const double *LF, int64_t n_pts,
                  const int64_t *p, const int64_t *seg_off, const int64_t *u_first,
                  uint64_t seed, double *d, int32_t *counts, int32_t nthreads)
{
    if (G < 1 || N < 1 || N > 64 || n_pts < 0 || !S || !LF || !seg_off || (n_pts && !p) || !d)
        return -1;
    for (int64_t k = 0; k < n_pts; ++k)
        if (p[k] < 0 || p[k] >= G || seg_off[k + 1] < seg_off[k] ||
            (u_first && u_first[k] < 0))
            return -1;
    struct fco_univ_ctx c = {N, S, LF, n_pts, p, seg_off, u_first, seed, d, counts};
    fco_parallel(n_pts, nthreads, fco_univ_task, &c);
    return 0;
}

/* ---- one matrix per universe (Algorithm 1 as printed), iterated (step 5) --- */
struct fco_fixed_ctx {
    int64_t G;
    int32_t N;
    const double *S, *F, *stat_diag;
    int32_t stat_mode;
    const double *d;
    const int64_t *p_idx;
    int32_t max_iter;
    double *dchi2, *chi2_min, *chi2_p;
    int64_t *argmin, *m_final;
    int32_t *iters;
    int failed;
};

static void fco_fixed_task(void *vctx, int64_t lo, int64_t hi)
{
    struct fco_fixed_ctx *c = (struct fco_fixed_ctx *)vctx;
    const int32_t N = c->N;
    double *A = (double *)malloc(sizeof(double) * N * N);
    double *L = (double *)malloc(sizeof(double) * N * N);
    if (!A || !L) {
        c->failed = 1;
        free(A);
        free(L);
        return;
    }
    for (int64_t k = lo; k < hi; ++k) {
        const double *dk = c->d + k * N;
        const int64_t p = c->p_idx[k];
        int64_t m = p;
        int32_t it = 0;
        double best, cp;
        int64_t qmin;
        for (;;) {
            /* M = Sigma_m^{-1}, used through the Cholesky factor of Sigma_m */
            fco_covariance(N, c->S + m * N, c->F, c->stat_mode, c->stat_diag, A);
            if (fco_cholesky(N, A, L) != 0) {
                c->failed = 1;
                break;
            }
            best = INFINITY;
            qmin = p;
            cp = NAN;
            for (int64_t q = 0; q < c->G; ++q) {
                const double v = fco_chi2(N, L, dk, c->S + q * N);
                if (q == p) cp = v;
                if (v < best) {
                    best = v;
                    qmin = q;
                }
            }
            if (it == c->max_iter || qmin == m) break;
            m = qmin;
            ++it;
        }
        c->dchi2[k] = cp - best;
        c->chi2_min[k] = best;
        c->argmin[k] = qmin;
        c->chi2_p[k] = cp;
        c->m_final[k] = m;
        c->iters[k] = it;
    }
    free(A);
    free(L);
}

int fco_scan_fixed_m(int64_t G, int32_t N, const double *S, const double *F, int32_t stat_mode,
                     const double *stat_diag, int64_t K, const double *d, const int64_t *p_idx,
                     int32_t max_iter, double *dchi2, double *chi2_min, int64_t *argmin,
                     double *chi2_p, int64_t *m_final, int32_t *iters, int32_t nthreads)
{
    if (G <= 0 || N <= 0 || N > 256 || !S || !F || K < 0 || max_iter < 0 ||
        (stat_mode == 1 && !stat_diag))
        return -1;
    if (K > 0 && (!d || !p_idx || !dchi2 || !chi2_min || !argmin || !chi2_p || !m_final || !iters))
        return -1;
    for (int64_t k = 0; k < K; ++k)
        if (p_idx[k] < 0 || p_idx[k] >= G) return -1;
    struct fco_fixed_ctx c = {G, N, S, F, stat_diag, stat_mode, d, p_idx, max_iter,
                              dchi2, chi2_min, chi2_p, argmin, m_final, iters, 0};
    fco_parallel(K, nthreads, fco_fixed_task, &c);
    return c.failed ? -2 : 0;
}
