/*
 * fc.h -- C ABI of the MI355X (gfx950) Feldman-Cousins grid-scan library.
 *
 * The library evaluates, for every pseudo-experiment ("universe") d drawn
 * around a true grid point p,
 *
 *     chi2(d, q) = (d - S(q))^T Sigma_q^{-1} (d - S(q))          (Eq. (1))
 *
 * at every point q of a D-dimensional grid, keeps the strict-"<" running
 * minimum over the grid in list order (Algorithm 1), forms
 *
 *     Delta chi2 = chi2(d, p) - min_q chi2(d, q)
 *
 * and reduces the Delta chi2 values of each true point to critical values
 * (Section 1, Figure 1: the value left of which a stated fraction of the
 * distribution lies) and a histogram.  The per-point covariance is the
 * statistical plus fractional-systematic form
 *
 *     Sigma_q = diag(stat_q) + F o (S(q) S(q)^T),  stat_q = S(q) (Pearson)
 *                                                  or a fixed vector.
 *
 * Conventions for every function:
 *   - Return value: FC_OK (0) or a negative fc_status.  fc_last_error()
 *     returns a thread-local, library-owned, NUL-terminated message
 *     describing the last failure on the calling thread.
 *   - "host" pointers are read only during the call.  "device" pointers are
 *     HIP device memory owned by the caller, read or written by work the call
 *     enqueues on `stream` (NULL = the null stream); that work is
 *     asynchronous unless stated otherwise.
 *   - Argument errors that can be seen on the host are reported before any
 *     device work is enqueued.  A device fault is reported as FC_ERR_DEVICE
 *     by the call that observes it.
 *   - A built grid is immutable: concurrent fc_scan calls on one grid from
 *     different streams are safe; fc_grid_destroy must not race with them.
 */
#ifndef FC_H
#define FC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fc_grid fc_grid; /* opaque, library-owned, device-resident */

enum fc_status_code {
    FC_OK = 0,
    FC_ERR_INVALID_ARG = -1, /* bad size, pointer, index or enum value        */
    FC_ERR_NOT_PD = -2,      /* a covariance is not positive definite         */
    FC_ERR_NOMEM = -3,       /* device or host allocation failed              */
    FC_ERR_DEVICE = -4,      /* a HIP call or kernel failed                   */
    FC_ERR_STATE = -5,       /* e.g. scanning with a form that was not built  */
    FC_ERR_UNSUPPORTED = -6  /* e.g. N > 64 bins                              */
};

/* Arithmetic forms of the scan (bit mask for fc_build_covariance). */
enum fc_form {
    FC_FORM_FP64 = 1,       /* FP64 factor, FP64 arithmetic                      */
    FC_FORM_FP32 = 2,       /* FP32 factor, FP32 MFMA contraction               */
    FC_FORM_SPLIT_BF16 = 4, /* hi+lo BF16 operands, FP32 MFMA accumulation      */
    FC_FORM_SPLIT_FP16 = 8  /* hi+lo FP16 operands, FP32 MFMA accumulation      */
};

enum fc_stat_mode {
    FC_STAT_PEARSON = 0, /* statistical term diag(S(q))                     */
    FC_STAT_FIXED = 1    /* statistical term diag(stat_diag), same for all q */
};

#define FC_MAX_BINS 64

/*
 * fc_build_grid -- make a grid resident on the current HIP device.
 *
 * Section 2: the D-dimensional rectangular grid is linearised into a list of
 * G = prod(axis_len) points, row-major with the LAST axis fastest:
 *     q = sum_d i_d * prod_{e>d} axis_len[e].
 * Section 1: every point carries a prediction S(q) of N bins; `central` is the
 * observed data vector c (optional, kept for the caller).
 *
 *   out        host out: receives the new handle (set to NULL on failure)
 *   D          1..16 axes
 *   axis_len   host [D], each >= 1; G must be < 2^31
 *   axis_vals  host [sum(axis_len)], the axes' values concatenated
 *   N          1..FC_MAX_BINS bins (larger N: FC_ERR_UNSUPPORTED)
 *   signal     host [G][N] FP64, row q = S(q); must be finite
 *   central    host [N] FP64 or NULL
 *   stream     stream for the uploads; the call synchronises it before returning
 * Ownership: the handle and all device memory behind it belong to the
 * library until fc_grid_destroy.
 */
int fc_build_grid(fc_grid **out, int32_t D, const int64_t *axis_len,
                  const double *axis_vals, int32_t N, const double *signal,
                  const double *central, hipStream_t stream);

/*
 * fc_build_covariance -- per-grid-point covariance, FP64 Cholesky and inverse
 * factor on the GPU, stored in the requested scan forms.
 *
 * For every q: Sigma_q = diag(stat_q) + F o (S(q) S(q)^T) (the inverse of
 * Sigma_q is the matrix M of Eq. (1)); L_q L_q^T = Sigma_q in FP64;
 * W_q = L_q^{-1} in FP64, so that Sigma_q^{-1} = W_q^T W_q and
 * chi2 = ||W_q (d - S(q))||^2.  W_q is stored in every form of `forms`.
 *
 *   g          grid from fc_build_grid (replaces any previously built forms)
 *   frac_cov   host [N][N] FP64 symmetric fractional systematic matrix F
 *   stat_mode  FC_STAT_PEARSON or FC_STAT_FIXED
 *   stat_diag  host [N] FP64 (FC_STAT_FIXED only, else ignored / NULL)
 *   forms      non-empty OR of fc_form values
 *   bad_q      host out: first q whose Sigma_q is not positive definite, or -1
 *   stream     the call synchronises this stream before returning
 * Returns FC_ERR_NOT_PD (with *bad_q set, no forms kept) if some Sigma_q has a
 * pivot <= 0 (or NaN) during the factorisation.
 */
int fc_build_covariance(fc_grid *g, const double *frac_cov, int32_t stat_mode,
                        const double *stat_diag, uint32_t forms, int64_t *bad_q,
                        hipStream_t stream);

/*
 * fc_scan -- Algorithm 1 for K universes on the GPU (asynchronous).
 *
 * For universe k with data d[k] and true point p_idx[k]:
 *   chi2_p[k]   = chi2(d[k], q = p_idx[k])            (Eq. (1) at the true point)
 *   chi2_min[k] = min over all q of chi2(d[k], q); the scan runs over q in
 *                 list order with a strict "<" starting from +inf, so among
 *                 exact ties the lowest q wins
 *   argmin[k]   = that q (p_idx[k] if no chi2 value is < +inf, e.g. NaN data)
 *   dchi2[k]    = chi2_p[k] - chi2_min[k]   (>= 0; the true point is scanned)
 * chi2 values are computed in the arithmetic of `form` (FP32 forms round each
 * chi2 to FP32; chi2_p and chi2_min are then exact FP64 copies of FP32
 * values, and dchi2 is their exact FP64 difference).
 *
 *   g        grid with `form` built (else FC_ERR_STATE)
 *   form     one fc_form value
 *   K        number of universes, 0 <= K <= 2^30 (K = 0 enqueues nothing)
 *   d        device [K][N] FP64, row-major
 *   p_idx    device [K] int64 true-point grid indices.  They live in device
 *            memory and are checked there, so that the call stays
 *            asynchronous: an index outside [0, G) gives that universe
 *            chi2_p = NaN and dchi2 = NaN (chi2_min and argmin as for any
 *            other universe) and touches no other memory.
 *   dchi2    device [K] FP64 output (required)
 *   chi2_min, chi2_p   device [K] FP64 outputs, each optional (NULL)
 *   argmin   device [K] int64 output, optional (NULL)
 * The FP32 and split forms keep the running minimum as packed (chi2, q) keys
 * in chi2_min's storage (decoded in place by the final pass), or, when
 * chi2_min is NULL, in a stream-ordered scratch of 8 K bytes; a NULL chi2_p
 * takes another 8 K bytes.  The FP64 form splits the grid into chunks when K
 * alone would leave CUs idle and merges their minima in grid order (the
 * same result); the chunk minima take a stream-ordered scratch of 16 bytes
 * per (chunk, universe), at most 2 GiB (chunks of 2048 grid points, longer
 * where that bound or the dispatch size would be passed).  Scratch is allocated with hipMallocAsync and
 * released with hipFreeAsync on `stream` (FC_ERR_NOMEM or FC_ERR_DEVICE if
 * that fails).
 * Universes with NaN/inf data get chi2_min = +inf, argmin = p, dchi2 = NaN;
 * other universes are unaffected.  The FP32 and split forms hold chi2 in
 * FP32: a chi2 value beyond FP32's range (about 3.4e38, residuals of order
 * 1e18) becomes +inf.  The split FP16 form keeps the universes at one
 * grid-wide power-of-two scale while their largest |d - o| (o the grid mean
 * of S) stays within 8x the grid's own spread of S - o, and gives a universe
 * beyond that its own power of two, so its FP16 operands stay finite.
 * Accuracy of the split forms: their products see d - o, not d - S_q, so the
 * chi2 error grows with R = max_j |d_j - o_j| / sqrt(S_p,j): about 2^-14 R
 * relative to max(1, chi2_p) for BF16 (within 1e-4 for R up to about 15, or
 * N in the tens of bins), about 2^5 times less for FP16.
 */
int fc_scan(const fc_grid *g, int32_t form, int64_t K, const double *d,
            const int64_t *p_idx, double *dchi2, double *chi2_min, int64_t *argmin,
            double *chi2_p, hipStream_t stream);

/*
 * fc_scan_no_alloc -- fc_scan for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, checks and results as fc_scan (bit for bit),
 * but the call allocates nothing: every scratch buffer the scan needs is
 * carved from a static device array of FC_NO_ALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on (from the first call on that
 * device until the process ends).  The FP32 and split forms need scratch
 * only for NULL outputs (8 K bytes for the keys when chi2_min is NULL, 8 K
 * when chi2_p is NULL); the FP64 form also keeps its chunk minima there,
 * with fewer grid chunks when they would not fit (the results do not depend
 * on the chunk count).  A call whose K needs more than the array holds
 * returns FC_ERR_INVALID_ARG before any device work.  Every call on one
 * device shares that device's array: calls that overlap in time on one
 * device (several streams or threads) race and must be serialised by the
 * caller; nothing is carried over between calls (what must start at zero is
 * cleared by each call's own kernels).
 */
#define FC_NO_ALLOC_SCRATCH_BYTES (32u << 20)
int fc_scan_no_alloc(const fc_grid *g, int32_t form, int64_t K, const double *d,
                     const int64_t *p_idx, double *dchi2, double *chi2_min, int64_t *argmin,
                     double *chi2_p, hipStream_t stream);

/*
 * fc_critical_value -- per-true-point critical values and histogram of
 * Delta chi2 (asynchronous).  Section 1 / Figure 1: the critical value for a
 * fraction alpha is the value left of which that fraction of the
 * distribution lies; it is taken as the type-1 order statistic
 *     crit = x_(j),  j = ceil(alpha * K_s) (IEEE FP64 product) clamped to [1, K_s],
 * of the K_s values of segment s sorted ascending with NaN last.
 *
 *   n_seg     number of segments (true points), >= 0
 *   seg_off   device [n_seg+1] int64 offsets into dchi2; segment s is
 *             dchi2[seg_off[s] .. seg_off[s+1]).  Checked on the device: a
 *             segment with negative or decreasing offsets yields NaN
 *             critical values and an all-zero histogram.
 *   dchi2     device FP64 values
 *   n_alpha   1..8 fractions, alpha host [n_alpha], each in (0, 1]
 *   crit      device out [n_seg][n_alpha] FP64 (NaN for an empty segment)
 *   n_bins    >= 1 (if hist != NULL)
 *   hist_hi   > 0: bin b < n_bins counts values with 0 <= x < hist_hi and
 *             floor(x / (hist_hi / n_bins)) = b (IEEE FP64, clamped to
 *             n_bins - 1); bin n_bins counts every other value, NaN included
 *   hist      device out [n_seg][n_bins+1] int64, or NULL for no histogram
 */
int fc_critical_value(int64_t n_seg, const int64_t *seg_off, const double *dchi2,
                      int32_t n_alpha, const double *alpha, double *crit, int32_t n_bins,
                      double hist_hi, int64_t *hist, hipStream_t stream);

/*
 * fc_scan_points -- the scan of fc_scan for universes grouped by true point,
 * the shape of Algorithm 1 (one true point p, N_univ universes fluctuated
 * around S(p)).  Segment s = [seg_off[s], seg_off[s+1]) holds universes of
 * true point p[s]; results are those of fc_scan with p_idx[u] = p[s] (to the
 * FP32 tolerance in the FP32 form, identical in the others).  The FP32 form
 * scans tiles of up to 256 universes of one segment with
 *     W_q (d - S_q) = W_q (d - S_p) + W_q (S_p - S_q),
 * d - S_p rounded to FP32 once and the second term taken from an offset
 * table built for the call (FP64 arithmetic, rounded once), so its grid loop
 * does no per-bin vector work.
 *   n_pts, p       n_pts >= 1 (when K > 0); device int64 [n_pts] true points;
 *                  a segment whose point is outside [0, G) is not scanned in
 *                  the FP32 form (dchi2, chi2_p NaN, chi2_min +inf, argmin p;
 *                  fc_scan's NaN in the others)
 *   seg_off        device int64 [n_pts+1], non-decreasing, seg_off[0] = 0,
 *                  seg_off[n_pts] = K (rows are assigned by it)
 *   K, d           host K; device [K][N] FP64 universes
 *   workspace      device scratch of at least fc_scan_points_workspace()
 *                  bytes, 256-byte aligned, owned by the caller; calls that
 *                  overlap in time need separate workspaces
 *   dchi2, chi2_min, argmin, chi2_p   as fc_scan (chi2_min, argmin and chi2_p
 *                  optional; the FP32 form then keeps its keys / chi2_p in
 *                  stream-ordered scratch of 8 K bytes each)
 * Asynchronous; FC_ERR_INVALID_ARG for a short or misaligned workspace.
 */
int fc_scan_points(const fc_grid *g, int32_t form, int64_t n_pts, const int64_t *p,
                   const int64_t *seg_off, int64_t K, const double *d, void *workspace,
                   size_t workspace_bytes, double *dchi2, double *chi2_min, int64_t *argmin,
                   double *chi2_p, hipStream_t stream);

/*
 * fc_scan_points_workspace -- bytes of workspace fc_scan_points needs for
 * (form, n_pts, K) on this grid: 8 K (+ alignment) and, for the FP32 form,
 * 16 ns n_pts G for the offset table (C2: 256 points: 614 MB).
 * FC_ERR_INVALID_ARG if that is beyond 2^60 bytes.
 */
int fc_scan_points_workspace(const fc_grid *g, int32_t form, int64_t n_pts, int64_t K,
                             size_t *bytes);

/*
 * Grid-sliced scans: Algorithm 1's loop over the grid cut into slices
 * [q0, q0 + nq) that run as separate calls -- one device's share when a grid
 * is sharded over devices, or pieces of a scan that should not hold the GPU
 * for its whole length.  Each universe carries a running state:
 *   keys[k]   uint64: (FP32 bit pattern of the smallest chi2 seen << 32) | its q,
 *             or the "none" value 0x7f800000ffffffff; chi2 >= 0, so the
 *             unsigned order of keys is the order of (chi2, q), and the minimum
 *             key is the strict-"<" running minimum of Algorithm 1 in list
 *             order (lowest q among exact ties)
 *   chi2_p[k] FP64: chi2(d[k], p[k]), written only by the slice that contains
 *             p[k]; 0 until then
 * Slices merge by a 64-bit unsigned MIN over keys and a SUM over chi2_p (every
 * universe's true point lies in exactly one slice), in any order and
 * grouping: slices that cover [0, G) once give, after fc_scan_state_finalize,
 * exactly the result of the one-call scan in the same form (FP32 and the
 * split forms; the FP64 form keeps FP64 minima and is not sliced:
 * FC_ERR_UNSUPPORTED).  Calls on one device may share one state (their
 * updates are atomic); calls on several devices keep their own states, merged
 * by those two reductions (an all-reduce MIN and SUM) before finalizing.
 */

/* fc_scan_state_init -- keys = none, chi2_p = 0 for K universes (device
 * arrays [K], caller-owned; 0 <= K <= 2^30).  Asynchronous. */
int fc_scan_state_init(int64_t K, uint64_t *keys, double *chi2_p, hipStream_t stream);

/*
 * fc_scan_slice -- fc_scan over the grid points [q0, q0 + nq) only, merged
 * into the state (keys, chi2_p).  Arguments as fc_scan; 0 <= q0, 0 <= nq,
 * q0 + nq <= G (else FC_ERR_INVALID_ARG); nq = 0 or K = 0 enqueue nothing.
 * form: FC_FORM_FP32 (the residual form of fc_scan) or a split form.
 * Asynchronous.
 */
int fc_scan_slice(const fc_grid *g, int32_t form, int64_t K, const double *d,
                  const int64_t *p_idx, int64_t q0, int64_t nq, uint64_t *keys, double *chi2_p,
                  hipStream_t stream);

/*
 * fc_scan_points_slice -- fc_scan_points over the grid points [q0, q0 + nq)
 * only, merged into the state (keys, chi2_p).  The FP32 form builds the
 * offset table for the slice's grid points; a segment whose point is outside
 * [0, G) is not scanned.  workspace: at least
 * fc_scan_points_slice_workspace(..., nq) bytes, 256-byte aligned.
 * Asynchronous.
 */
int fc_scan_points_slice(const fc_grid *g, int32_t form, int64_t n_pts, const int64_t *p,
                         const int64_t *seg_off, int64_t K, const double *d, int64_t q0,
                         int64_t nq, void *workspace, size_t workspace_bytes, uint64_t *keys,
                         double *chi2_p, hipStream_t stream);

/* fc_scan_points_slice_workspace -- as fc_scan_points_workspace with the
 * offset table sized for nq grid points (0 <= nq <= G): 8 K (+ alignment) and,
 * for the FP32 form, 16 ns n_pts nq bytes. */
int fc_scan_points_slice_workspace(const fc_grid *g, int32_t form, int64_t n_pts, int64_t K,
                                   int64_t nq, size_t *bytes);

/*
 * fc_scan_state_finalize -- the outputs of fc_scan from a merged state:
 * chi2_min[k] = the FP32 chi2 of keys[k] (+inf for none), argmin[k] = its q
 * (p_idx[k] for none), dchi2[k] = chi2_p[k] - chi2_min[k], NaN for none and
 * for a true point p_idx[k] outside [0, G) (whose chi2_p no slice writes).
 *   p_idx    device [K] int64, required (the universes' true points)
 *   keys, chi2_p   device [K] merged state (read only)
 *   dchi2, chi2_min   device out [K] FP64; argmin device out [K] int64
 * Asynchronous.
 */
int fc_scan_state_finalize(const fc_grid *g, int64_t K, const int64_t *p_idx,
                           const uint64_t *keys, const double *chi2_p, double *dchi2,
                           double *chi2_min, int64_t *argmin, hipStream_t stream);

/*
 * fc_scan_fixed_m -- Algorithm 1 as printed: one matrix M for the whole grid
 * scan of a universe, and its iteration (Section 2, step 5: update M at the
 * minimiser and scan again until the minimiser repeats).  Per universe k,
 * M = Sigma_m^{-1} with m = p_idx[k] first; after a scan with minimiser
 * q_min != m (and fewer than max_iter re-scans done) m = q_min and the
 * universe is scanned again.  With the last M:
 *     chi2(d, q) = (d - S_q)^T M (d - S_q)   for every q (min: strict "<" in
 *     grid order, lowest q among equal values),  dchi2 = chi2(d, S_p) - min.
 * max_iter = 0 is the fixed-matrix scan.  FP64 (needs FC_FORM_FP64): chi2 is
 * formed as |y|^2 + |t_q|^2 - 2 y.t_q in the space whitened by W_m, the cross
 * term on the FP64 matrix cores.
 *   d, p_idx   device [K][N] FP64, [K] int64 (0 <= p < G, else FC_ERR_INVALID_ARG)
 *   dchi2, chi2_min, chi2_p  device out [K] FP64; argmin device out [K] int64
 *   m_final    device out [K] int64 (the m of the last scan), or NULL
 *   iters      device out [K] int32 (re-scans done), or NULL
 * K <= 2^30, 0 <= max_iter <= 64.  Synchronous (universes are grouped by m
 * on the host between scans).
 */
int fc_scan_fixed_m(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                    int32_t max_iter, double *dchi2, double *chi2_min, int64_t *argmin,
                    double *chi2_p, int64_t *m_final, int32_t *iters, hipStream_t stream);

/*
 * fc_generate_universes -- draw universes on the device (Section 2, steps 1
 * and 2 of the per-universe procedure: the prediction at the true point is
 * fluctuated into fake data).  Row r in [seg_off[k], seg_off[k+1]) is universe
 * j = u_first[k] + (r - seg_off[k]) of true point p[k]:
 *     d[r][i] = n_i + S_p[i] * sum_{l <= i} L_F[i][l] g_l,
 *     n_i ~ Poisson(S_p[i]),  g ~ N(0, I),  L_F = chol(F),
 * so Cov(d) = diag(S_p) + F o (S_p S_p^T), the covariance of the scan.
 * Random numbers: Philox4x64-10 (Salmon et al., SC'11) with key (seed, 0);
 * block b of purpose t (0 Poisson, 1 normal) for (p, j, bin i) has counter
 * (j, p, i << 32 | t << 28 | b, 0); word w -> uniform ((w >> 11) + 0.5) 2^-53.
 * Poisson: multiplication method below mean 10, Hormann's PTRS from 10 up;
 * normal: Box-Muller from the bin's normal block.  A universe depends only on
 * (seed, p, j): any split into calls or batches gives identical rows.
 *   n_pts, p       device int64 [n_pts] true points (outside [0, G): rows NaN,
 *                  p_idx -1, counts -1)
 *   seg_off        device int64 [n_pts+1], non-decreasing, seg_off[0] = 0,
 *                  seg_off[n_pts] = K (rows are assigned by it)
 *   u_first        device int64 [n_pts] first universe index, or NULL (all 0)
 *   K              host: number of rows
 *   d              device out [K][N] FP64
 *   p_idx          device out [K] int64 (the row's true point), or NULL
 *   counts         device out [K][N] int32 (the Poisson parts), or NULL
 * Needs fc_build_covariance (FC_ERR_STATE) with F positive definite
 * (FC_ERR_NOT_PD).  Asynchronous.
 */
int fc_generate_universes(const fc_grid *g, int64_t n_pts, const int64_t *p,
                          const int64_t *seg_off, const int64_t *u_first, uint64_t seed,
                          int64_t K, double *d, int64_t *p_idx, int32_t *counts,
                          hipStream_t stream);

/*
 * fc_region -- Feldman-Cousins confidence region with per-point universe
 * counts.  Section 2 builds the Delta chi^2 distribution of every true point
 * from universes drawn at it; the paper's closing section proposes letting
 * the universe count differ per point so that large counts go only to points
 * near the eventual contour.  In rounds, on the device:
 *   - every point starts with K0 universes (fc_generate_universes' stream,
 *     universe indices 0 .. K0-1, this seed), scanned in `form`;
 *   - per point: crit[a] = x_(ceil(alpha_a K)) over its K values, and the band
 *     [x_(j - delta), x_(j + delta)], j = ceil(alpha_a K), delta =
 *     ceil(z sqrt(K alpha_a (1 - alpha_a))), ranks clamped to [1, K];
 *   - a point whose data value dchi2_data[p] lies inside some band is
 *     undecided; undecided points below K_max double K (universes K .. 2K-1,
 *     at most K_max) and the round repeats until none is left to refine.
 * Then accepted[k][a] = dchi2_data[p_k] <= crit[k][a] (NaN: not accepted).
 *   pts          host [n_pts] grid indices, or NULL with n_pts = G (every point)
 *   K0, K_max    1 <= K0 <= K_max <= 2^24; z >= 0 (band half-width in sigmas)
 *   n_alpha      1..4 fractions in (0, 1] (host)
 *   dchi2_data   device [G] from fc_data_scan
 *   crit         device out [n_pts][n_alpha] FP64
 *   accepted     device out [n_pts][n_alpha] uint8
 *   K_used       host out [n_pts]: universes each point ended with
 *   n_rounds, n_evals  host out: rounds run, universe x grid-point evaluations
 * Needs the form built and F positive definite (fc_generate_universes).
 * Device memory: n_pts * K_max doubles plus a batch of 2^19 universes.
 * Synchronous (the refinement decisions are taken on the host).
 */
int fc_region(const fc_grid *g, int32_t form, int64_t n_pts, const int64_t *pts, int64_t K0,
              int64_t K_max, double z, uint64_t seed, int32_t n_alpha, const double *alpha,
              const double *dchi2_data, double *crit, uint8_t *accepted, int64_t *K_used,
              int32_t *n_rounds, double *n_evals, hipStream_t stream);

/*
 * fc_data_scan -- the observed-data statistic (Section 1: the scan looks for
 * the points compatible with the central data vector c; Algorithm 1's inner
 * loop run once with c as the data):
 *     dchi2_data[q] = chi2(c, q) - min_q' chi2(c, q')     for every q,
 * in FP64 with the FP64 factor (needs FC_FORM_FP64, else FC_ERR_STATE).
 *   central    host [N] FP64, or NULL for the vector given to fc_build_grid
 *              (FC_ERR_STATE if there is none)
 *   dchi2_data device out [G] FP64
 *   chi2_min   host out: the minimum over the grid (NaN if every chi2 is NaN)
 *   argmin     host out: the lowest q reaching it (-1 if all chi2 are NaN)
 * Synchronises `stream`.
 */
int fc_data_scan(const fc_grid *g, const double *central, double *dchi2_data, double *chi2_min,
                 int64_t *argmin, hipStream_t stream);

/*
 * fc_acceptance -- Feldman-Cousins acceptance of true points (Section 1):
 *     accepted[k] = dchi2_data[p[k]] <= crit[k * crit_stride]
 * (asynchronous).  p device [n_pts] int64 (outside [0, G): not accepted),
 * crit device (e.g. one column of fc_critical_value's output, stride n_alpha),
 * dchi2_data device [G] from fc_data_scan, accepted device out [n_pts] uint8.
 */
int fc_acceptance(const fc_grid *g, int64_t n_pts, const int64_t *p, const double *crit,
                  int64_t crit_stride, const double *dchi2_data, uint8_t *accepted,
                  hipStream_t stream);

/*
 * fc_grid_inverse_cov -- write Sigma_q^{-1} = W_q^T W_q (FP64, from the FP64
 * factor) for q = q0 .. q0+nq-1 into device out [nq][N][N] (asynchronous).
 * Needs FC_FORM_FP64 built (else FC_ERR_STATE).
 */
int fc_grid_inverse_cov(const fc_grid *g, int64_t q0, int64_t nq, double *out,
                        hipStream_t stream);

/* fc_grid_info -- sizes of a grid (any out pointer may be NULL). */
int fc_grid_info(const fc_grid *g, int32_t *D, int32_t *N, int64_t *G, uint32_t *forms);

/* fc_grid_device_bytes -- device memory held by the grid (0 for NULL). */
size_t fc_grid_device_bytes(const fc_grid *g);

/* fc_grid_destroy -- free a grid and its device memory (NULL is a no-op).
 * Synchronises the device before freeing. */
void fc_grid_destroy(fc_grid *g);

/* fc_last_error -- message of the last failure on this thread ("" if none). */
const char *fc_last_error(void);

/*
 * Kernel timing for measurement tools (no paper passage: instrumentation).
 * fc_profile_enable(1) clears earlier records and starts bracketing every
 * launch of the scan kernels (k_scan_f64m, k_scan_fp32, k_scan_fp32_pts,
 * k_offset_table, k_scan_split) and of the covariance build (k_cov_build)
 * with two HIP events recorded on the stream the
 * kernel is launched on; fc_profile_enable(0) stops (records are kept).
 * fc_profile_read waits for the recorded launches of one kernel and returns
 * their count and summed duration in milliseconds.  Thread-safe; profiling
 * adds two event records per launch.
 */
int fc_profile_enable(int32_t on);
int fc_profile_read(const char *kernel, int64_t *launches, double *total_ms);

/* ------------------------------------------------------------------------
 * Serving: FC requests against resident grids, with continuous batching.
 *
 * A request is one true point p of one resident grid and K universes
 * (Section 2: the Delta chi2 distribution of a single point from N_univ
 * fluctuated universes; Algorithm 1 for that point).  Its result is what
 * fc_scan + fc_critical_value give for the same inputs, bit for bit: the
 * server only changes which launch and which block evaluate each
 * (universe, grid point) pair, and the running minimum is merged in an
 * order-independent way.
 *
 * A scheduler thread owned by the server admits queued requests in arrival
 * order while their device memory fits a fixed budget (allocated once at
 * creation), uploads their universes, and keeps a short queue of batched
 * launches per bin-count class: every launch takes work items (a tile of
 * universes x a range of grid points) from all admitted requests in turn, so
 * requests that arrive while others run join the next launch and their work
 * overlaps on the device.  A request's Delta chi2 values, critical values
 * and histogram are copied back when its last item has run.
 * ------------------------------------------------------------------------ */
typedef struct fc_server fc_server; /* opaque, library-owned */

enum fc_server_policy {
    FC_SCHED_FAIR = 0,  /* every admitted request gets a slice of each launch (round robin) */
    FC_SCHED_FIFO = 1   /* the oldest request takes all it can use, younger ones backfill   */
};

enum fc_request_state {
    FC_REQ_QUEUED = 0,   /* waiting for device memory                  */
    FC_REQ_RUNNING = 1,  /* admitted; items queued or running          */
    FC_REQ_DONE = 2,     /* results are on the host                    */
    FC_REQ_FAILED = -1   /* a device error ended it (see fc_last_error) */
};

/*
 * fc_server_create -- start a server over resident grids.
 *
 *   out          host out: the new server
 *   grids        host [n_grids] grid handles, each with `form` built; the
 *                caller keeps them alive until fc_server_destroy returns
 *   form         one fc_form value other than FC_FORM_FP64
 *   hbm_budget   bytes of device memory for request data (universes,
 *                outputs), allocated once; requests are admitted while they fit
 *   host_budget  bytes of page-locked host memory for staging and results
 *   n_alpha, alpha, n_bins, hist_hi   critical-value settings applied to every
 *                request (as in fc_critical_value; n_bins >= 1)
 *   launch_evals target (universe x grid point) evaluations per batched
 *                launch; 0 selects a default (1.5e8 FP32, 4.5e8 split forms)
 *   policy       FC_SCHED_FAIR or FC_SCHED_FIFO: how a launch's work is shared
 *                among the admitted requests
 */
int fc_server_create(fc_server **out, const fc_grid *const *grids, int32_t n_grids, int32_t form,
                     size_t hbm_budget, size_t host_budget, int32_t n_alpha, const double *alpha,
                     int32_t n_bins, double hist_hi, double launch_evals, int32_t policy);

/*
 * fc_server_submit -- queue one request (returns at once).
 *   grid   index into the server's grids;  p   true point, 0 <= p < G
 *   K      1..2^20 universes;  d   host [K][N] FP64, copied during the call
 *   req    host out: request id
 * FC_ERR_NOMEM if the request alone exceeds hbm_budget or the host staging
 * memory is exhausted.
 */
int fc_server_submit(fc_server *s, int32_t grid, int64_t p, int64_t K, const double *d,
                     int64_t *req);

/*
 * fc_server_submit_drawn -- queue one request whose K universes are drawn on
 * the device at admission (Section 2, steps 1 and 2 of the per-universe
 * procedure): universes u_first .. u_first+K-1 of true point p with `seed`,
 * the stream of fc_generate_universes.  Results are bitwise those of
 * fc_server_submit with the same universes uploaded; only the outputs cross
 * PCIe.
 *   u_first >= 0;  other arguments as fc_server_submit.
 * FC_ERR_NOT_PD if the grid's fractional matrix has no Cholesky factor.
 */
int fc_server_submit_drawn(fc_server *s, int32_t grid, int64_t p, int64_t K, uint64_t seed,
                           int64_t u_first, int64_t *req);

/*
 * fc_server_poll -- state of a request; when FC_REQ_DONE, copies its results
 * into the non-NULL host buffers: dchi2, chi2_min, chi2_p [K] FP64, argmin [K]
 * int64, crit [n_alpha] FP64, hist [n_bins+1] int64, and latency (seconds from
 * submit to results on the host).  release != 0 with a done request frees its
 * host storage (the id is then unknown).
 */
int fc_server_poll(fc_server *s, int64_t req, int32_t *state, double *dchi2, double *chi2_min,
                   int64_t *argmin, double *chi2_p, double *crit, int64_t *hist, double *latency,
                   int32_t release);

/* fc_server_stats -- totals so far (any out pointer may be NULL): requests
 * done, launches, evaluations, device bytes in use. */
int fc_server_stats(fc_server *s, int64_t *done, int64_t *launches, double *evals,
                    size_t *hbm_in_use);

/* fc_server_destroy -- stop admitting, wait for the launches already on the
 * device, drop requests not yet done, free everything (NULL is a no-op). */
void fc_server_destroy(fc_server *s);

#ifdef __cplusplus
}
#endif
#endif /* FC_H */
