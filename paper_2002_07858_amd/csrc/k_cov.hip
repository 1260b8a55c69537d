// k_cov.hip -- per-grid-point covariance, FP64 Cholesky and inverse factor.
//
// For grid point q (Section 1: M in Eq. (1) is the inverse of a covariance
// carrying statistical and systematic uncertainties):
//     Sigma_q = diag(stat_q) + F o (S_q S_q^T)
//     L_q L_q^T = Sigma_q          right-looking Cholesky, FP64, in LDS
//     W_q = L_q^{-1}               column-wise forward substitution, FP64
// so that Sigma_q^{-1} = W_q^T W_q and chi2 = ||W_q r||^2.  This is the step
// whose conditioning needs FP64; the scan forms only ever see W_q.
//
// One wave (64 lanes) per grid point: lane i owns row i during the Cholesky
// and column i during the inversion.  A non-positive (or NaN) pivot marks the
// point as not positive definite.  L and W share one LDS matrix: L in the
// lower triangle, W_q's column c transposed into the strict upper part of row
// c and its diagonal into a spare last column (28 KB per point at N = 57, so
// five points fit a CU's LDS at once; 13 KB at N = 38).
#include "fc_internal.h"

namespace fcx {

// Row stride of the LDS matrix: N + 1 rounded up to an odd count of doubles
// (consecutive rows then start on different bank pairs); its last column holds
// W_q's diagonal.
__host__ __device__ inline int cov_ld(int N) { return (N + 1) | 1; }

// LDS bytes of one point: the N x ld matrix, then column j of L, S_q - fl32(S_q)
// and S_q - o.
inline size_t cov_lds_bytes(int N)
{
    return sizeof(double) * ((size_t)N * cov_ld(N) + 3 * kMaxBins);
}

// W_q[r][c] (r >= c) from the shared matrix.
__device__ inline double wget(const double *A, int ld, int r, int c)
{
    return (r == c) ? A[c * ld + ld - 1] : A[c * ld + r];
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// hi + lo split of eight FP32 values into two 16-byte fragments (round to
// nearest even for both halves).
template <bool FP16>
__device__ inline void split8(const float (&x)[8], uint4 &hi, uint4 &lo)
{
    if constexpr (FP16) {
        f16x8 h, l;
        for (int e = 0; e < 8; ++e) {
            h[e] = (_Float16)x[e];
            l[e] = (_Float16)(x[e] - (float)h[e]);
        }
        hi = __builtin_bit_cast(uint4, h);
        lo = __builtin_bit_cast(uint4, l);
    } else {
        bf16x8 h, l;
        for (int e = 0; e < 8; ++e) {
            h[e] = (__bf16)x[e];
            l[e] = (__bf16)(x[e] - (float)h[e]);
        }
        hi = __builtin_bit_cast(uint4, h);
        lo = __builtin_bit_cast(uint4, l);
    }
}

// One split-form record (see fc_internal.h) from the FP64 factor in LDS.
template <bool FP16>
__device__ void write_split_record(const double *A, int ld, const double *sdo, int N, int ed,
                                   uint4 *rq)
{
    const int i = threadIdx.x;
    const int nk = split_nk(N), nb = split_nb(N);
    // per-point power-of-two scale of the factor (FP16 range)
    int eq = 0;
    if constexpr (FP16) {
        double wm = 0.0;
        if (i < N)
            for (int r = i; r < N; ++r) wm = fmax(wm, fabs(wget(A, ld, r, i)));
        for (int m = 32; m > 0; m >>= 1) wm = fmax(wm, __shfl_xor(wm, m));
        eq = (wm > 0.0) ? 13 - ilogb(wm) : 0;
    }
    // fragments of every (k-step, row block) pair
    for (int s = 0; s < nk; ++s) {
        for (int b = 2 * s; b < nb; ++b) {
            const int t = split_pair_index(nk, nb, s, b);
            const int rr = 16 * b + (i & 15), c0 = 32 * s + 8 * (i >> 4);
            float x[8];
            for (int e = 0; e < 8; ++e) {
                const int cc = c0 + e;
                x[e] = (rr < N && cc <= rr) ? (float)ldexp(wget(A, ld, rr, cc), eq) : 0.0f;
            }
            uint4 hi, lo;
            split8<FP16>(x, hi, lo);
            rq[t * 128 + i] = hi;
            rq[t * 128 + 64 + i] = lo;
        }
    }
    // u_q = W_q (S_q - o) in FP64, in the accumulator's row order [g][b][j]
    {
        const int g = i >> 4, b = (i >> 2) & 3, j = i & 3;
        const int row = 16 * b + 4 * g + j;
        double u = 0.0;
        if (row < N) {
#pragma unroll 4
            for (int k = 0; k <= row; ++k) u += wget(A, ld, row, k) * sdo[k];
        }
        reinterpret_cast<float *>(rq + split_u_unit(nk, nb))[i] = (float)ldexp(-u, eq + ed);
    }
    const int su = split_scale_unit(nk, nb), ru = split_rec_units(nk, nb);
    if (i == 0) rq[su] = make_uint4(__float_as_uint(ldexpf(1.0f, -2 * (eq + ed))), 0u, 0u, 0u);
    for (int u = su + 1 + i; u < ru; u += 64) rq[u] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ __launch_bounds__(64) void k_cov_build(
    const double *__restrict__ S64, const double *__restrict__ F, const double *__restrict__ stat,
    const double *__restrict__ off, int N, int64_t G, int stat_mode, uint32_t forms, int ns,
    int ed16, double *__restrict__ W64, uint4 *__restrict__ R64, uint4 *__restrict__ R32,
    uint4 *__restrict__ RB16, uint4 *__restrict__ RH16, unsigned long long *__restrict__ bad_q)
{
    extern __shared__ double smem[];
    const int ld = cov_ld(N);
    // disjoint pieces of the block's LDS (restrict: the trailing update's loads
    // of colj are not ordered behind its stores to A)
    double *__restrict__ A = smem;               // [N][ld]: L, W^T above it, W's diagonal last
    double *__restrict__ colj = A + N * ld;      // column j of L
    double *__restrict__ sdl = colj + kMaxBins;  // S_q - fl32(S_q)
    double *__restrict__ sdo = sdl + kMaxBins;   // S_q - o
    const int i = threadIdx.x;
    const double stat_i = (i < N && stat_mode != FC_STAT_PEARSON) ? stat[i] : 0.0;

    for (int64_t q = blockIdx.x; q < G; q += gridDim.x) {
        const double *Sq = S64 + q * N;
        // ---- Sigma_q, row i ------------------------------------------------
        const double si = (i < N) ? Sq[i] : 0.0;
        if (i < N) {
#pragma unroll 8
            for (int j = 0; j < N; ++j) A[i * ld + j] = F[i * N + j] * (si * Sq[j]);
        }
        if (i < N) {
            A[i * ld + i] += (stat_mode == FC_STAT_PEARSON) ? si : stat_i;
            sdl[i] = si - (double)(float)si;
            sdo[i] = si - off[i];
        }
        __syncthreads();

        // ---- right-looking Cholesky ----------------------------------------
        bool ok = true;
        for (int j = 0; j < N; ++j) {
            const double piv = A[j * ld + j];
            if (!(piv > 0.0)) {  // uniform: every lane read the same pivot
                ok = false;
                break;
            }
            const double ljj = sqrt(piv);
            __syncthreads();
            double lij = 0.0;
            if (i == j) A[j * ld + j] = ljj;
            if (i > j && i < N) {
                lij = A[i * ld + j] / ljj;
                A[i * ld + j] = lij;
                colj[i] = lij;
            }
            __syncthreads();
            // lane i updates its own row from the column copy: the loads come
            // from another array than the stores, so they can be issued ahead
            if (i > j && i < N) {
                double *__restrict__ row = A + i * ld;
                int k = j + 1;
                for (; k + 3 <= i; k += 4) {  // four loads of each array, then the stores
                    const double c0 = colj[k], c1 = colj[k + 1], c2 = colj[k + 2],
                                 c3 = colj[k + 3];
                    const double a0 = row[k], a1 = row[k + 1], a2 = row[k + 2], a3 = row[k + 3];
                    row[k] = a0 - lij * c0;
                    row[k + 1] = a1 - lij * c1;
                    row[k + 2] = a2 - lij * c2;
                    row[k + 3] = a3 - lij * c3;
                }
                for (; k <= i; ++k) row[k] -= lij * colj[k];
            }
            __syncthreads();
        }
        if (!ok) {
            if (i == 0) atomicMin(bad_q, (unsigned long long)q);
            __syncthreads();
            continue;
        }

        // ---- W = L^{-1}: lane c solves L w = e_c for its own column ----------
        // (w[k] = 0 for k < c, so the sums start at k = c; the stores go to row
        // c's strict upper part and its spare column, which no other lane reads)
        const int c = i;
        if (c < N) {
            A[c * ld + ld - 1] = 1.0 / A[c * ld + c];
            for (int r = c + 1; r < N; ++r) {
                double acc = 0.0;
#pragma unroll 4
                for (int k = c; k < r; ++k) acc -= A[r * ld + k] * wget(A, ld, k, c);
                A[c * ld + r] = acc / A[r * ld + r];
            }
        }
        __syncthreads();

        // ---- store the requested forms -------------------------------------
        if (forms & FC_FORM_FP64) {
            double *Wq = W64 + q * ((int64_t)N * (N + 1) / 2);
            if (c < N)
                for (int r = c; r < N; ++r) Wq[tri_index(r, c)] = wget(A, ld, r, c);
        }
        if (forms & FC_FORM_FP64) {
            // tile records of the FP64 MFMA form: element e of the record is
            // (pair, position, tile of the pair), then the signal and the lead
            // columns in the order the scan's lanes read them
            const int nb = f64_nb(N), nt = f64_ntile(N), P = f64_pad(N), nbe = f64_nbe(N);
            const int sig = f64_sig_double(N), lead = f64_lead_double(N), nl = f64_lead(N);
            double *rq = reinterpret_cast<double *>(R64 + q * (int64_t)f64_rec_units(N));
            for (int e = i; e < sig; e += 64) {
                const int t = 2 * (e >> 5) + (e & 1), pos = (e >> 1) & 15;
                double val = 0.0;
                if (t < nt) {
                    const int rr = 4 * f64_tile_r(N, t) + (pos & 3) - P;
                    const int cc = 4 * f64_tile_kb(N, t) + (pos >> 2) - P;
                    if (rr >= 0 && rr < N && cc >= 0 && cc <= rr) val = wget(A, ld, rr, cc);
                }
                rq[e] = val;
            }
            for (int e = i; e < 4 * nbe; e += 64) {
                const int g = e / nbe, r = e % nbe, k = 4 * r + g - P;
                rq[sig + e] = (k >= 0 && k < N) ? Sq[k] : 0.0;
            }
            for (int e = i; e < 4 * nbe * nl; e += 64) {
                const int c = e / (4 * nbe), g = (e / nbe) % 4, r = e % nbe;
                const int rr = 4 * r + g - P;
                rq[lead + e] = (r < nb && rr >= c && rr < N) ? wget(A, ld, rr, c) : 0.0;
            }
        }
        if (forms & FC_FORM_FP32) {
            // A register v, lane i = 4 X + m: pair t = 16 v + X, i.e. padded
            // row 4b + m and padded bin k' of that pair
            const int ru = rec_units(ns), wu = rec_w_units(ns);
            const int P = fp32_pad(ns, N), np = fp32_npairs(ns);
            uint4 *rq = R32 + q * (int64_t)ru;
            float *Wq = reinterpret_cast<float *>(rq);
            const int X = i >> 2, m = i & 3;
            for (int v = 0; v < 4 * n_groups_from_ns(ns); ++v) {
                const int t = 16 * v + X;
                float val = 0.0f;
                if (t < np) {
                    const int kp = fp32_pair_kp(ns, t), b = fp32_pair_b(ns, t);
                    const int rr = 4 * b + m - P, cc = kp - P;
                    if (rr >= 0 && rr < N && cc >= 0 && cc <= rr) val = (float)wget(A, ld, rr, cc);
                }
                Wq[((v >> 2) * 64 + i) * 4 + (v & 3)] = val;
            }
            // FP32 part of the signal (real bin order), then minus W_q times
            // its rounding error (padded row order)
            float *Sp = reinterpret_cast<float *>(rq + wu);
            {
                Sp[i] = (i < N) ? (float)Sq[i] : 0.0f;
                const int rr = i - P;
                double cv = 0.0;
                if (rr >= 0 && rr < N) {
#pragma unroll 4
                    for (int kk = 0; kk <= rr; ++kk) cv -= wget(A, ld, rr, kk) * sdl[kk];
                }
                Sp[64 + i] = (float)cv;
            }
        }
        if (forms & (FC_FORM_SPLIT_BF16 | FC_FORM_SPLIT_FP16)) {
            const int64_t sru = split_rec_units(split_nk(N), split_nb(N));
            if (forms & FC_FORM_SPLIT_BF16)
                write_split_record<false>(A, ld, sdo, N, 0, RB16 + q * sru);
            if (forms & FC_FORM_SPLIT_FP16)
                write_split_record<true>(A, ld, sdo, N, ed16, RH16 + q * sru);
        }
        __syncthreads();
    }
}

hipError_t launch_cov_build(const fc_grid *g, const double *F, const double *stat, int stat_mode,
                            uint32_t forms, double *W64, uint4 *R64, uint4 *R32, uint4 *RB16,
                            uint4 *RH16, unsigned long long *bad_q, hipStream_t st)
{
    const int64_t blocks = g->G < 65536 ? g->G : 65536;
    hipLaunchKernelGGL(k_cov_build, dim3((unsigned)blocks), dim3(64), cov_lds_bytes(g->N), st,
                       g->S64, F, stat,
                       g->off, g->N, g->G, stat_mode, forms, g->ns, g->ed16, W64, R64, R32, RB16,
                       RH16, bad_q);
    return hipGetLastError();
}

// Sigma_q^{-1} = W_q^T W_q from the FP64 factor; one block per grid point,
// thread (i, j) -> out[i][j] = sum_{r >= max(i,j)} W[r][i] W[r][j].
__global__ __launch_bounds__(256) void k_inverse_cov(const double *__restrict__ W64, int N,
                                                    int64_t q0, int64_t nq,
                                                    double *__restrict__ out)
{
    const int64_t qq = blockIdx.x;
    if (qq >= nq) return;
    const double *Wq = W64 + (q0 + qq) * ((int64_t)N * (N + 1) / 2);
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        const int lo = i > j ? i : j;
        double acc = 0.0;
        for (int r = lo; r < N; ++r) acc += Wq[tri_index(r, i)] * Wq[tri_index(r, j)];
        out[qq * N * N + e] = acc;
    }
}

hipError_t launch_inverse_cov(const fc_grid *g, int64_t q0, int64_t nq, double *out,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_inverse_cov, dim3((unsigned)nq), dim3(256), 0, st, g->W64, g->N, q0, nq,
                       out);
    return hipGetLastError();
}

}  // namespace fcx
