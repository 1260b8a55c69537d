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
// point as not positive definite.
#include "fc_internal.h"

namespace fcx {

constexpr int kLdsStride = kMaxBins + 1;

__global__ __launch_bounds__(64) void k_cov_build(
    const double *__restrict__ S64, const double *__restrict__ F, const double *__restrict__ stat,
    int N, int64_t G, int stat_mode, uint32_t forms, int ns, double *__restrict__ W64,
    uint4 *__restrict__ R32, unsigned long long *__restrict__ bad_q)
{
    __shared__ double A[kMaxBins * kLdsStride];
    __shared__ double Wc[kMaxBins * kLdsStride];
    const int i = threadIdx.x;
    const int nb = n_rowblocks_from_ns(ns);

    for (int64_t q = blockIdx.x; q < G; q += gridDim.x) {
        const double *Sq = S64 + q * N;
        // ---- Sigma_q, row i ------------------------------------------------
        const double si = (i < N) ? Sq[i] : 0.0;
        for (int j = 0; j < N; ++j) {
            double v = 0.0;
            if (i < N) {
                v = F[i * N + j] * (si * Sq[j]);
                if (i == j) v += (stat_mode == FC_STAT_PEARSON) ? si : stat[i];
            }
            A[i * kLdsStride + j] = v;
        }
        __syncthreads();

        // ---- right-looking Cholesky ----------------------------------------
        bool ok = true;
        for (int j = 0; j < N; ++j) {
            const double piv = A[j * kLdsStride + j];
            if (!(piv > 0.0)) {  // uniform: every lane read the same pivot
                ok = false;
                break;
            }
            const double ljj = sqrt(piv);
            __syncthreads();
            if (i == j) A[j * kLdsStride + j] = ljj;
            if (i > j && i < N) A[i * kLdsStride + j] = A[i * kLdsStride + j] / ljj;
            __syncthreads();
            if (i > j && i < N) {
                const double lij = A[i * kLdsStride + j];
                for (int k = j + 1; k <= i; ++k)
                    A[i * kLdsStride + k] -= lij * A[k * kLdsStride + j];
            }
            __syncthreads();
        }
        if (!ok) {
            if (i == 0) atomicMin(bad_q, (unsigned long long)q);
            __syncthreads();
            continue;
        }

        // ---- W = L^{-1}: lane c solves L w = e_c for its own column ----------
        const int c = i;
        for (int r = 0; r < N; ++r) {
            double acc = (r == c) ? 1.0 : 0.0;
            for (int k = 0; k < r; ++k) acc -= A[r * kLdsStride + k] * Wc[k * kLdsStride + c];
            Wc[r * kLdsStride + c] = (c < N && r >= c) ? acc / A[r * kLdsStride + r] : 0.0;
        }
        __syncthreads();

        // ---- store the requested forms -------------------------------------
        if (forms & FC_FORM_FP64) {
            double *Wq = W64 + q * ((int64_t)N * (N + 1) / 2);
            if (c < N)
                for (int r = c; r < N; ++r) Wq[tri_index(r, c)] = Wc[r * kLdsStride + c];
        }
        if (forms & FC_FORM_FP32) {
            // pair t = (s, b) in the scan's order; lane i holds W[16b + i%16 - r0][4s + i/16]
            const int ru = rec_units(ns), wu = rec_w_units(ns);
            uint4 *rq = R32 + q * (int64_t)ru;
            float4 *Wq = reinterpret_cast<float4 *>(rq);
            const int row_in = i & 15, col_in = i >> 4;
            const int r0 = row_shift(ns);
            float vals[4];
            int slot = 0, gi = 0;
            for (int s = 0; s < ns; ++s) {
                for (int b = first_block_of_kstep(ns, s); b < nb; ++b) {
                    const int rr = 16 * b + row_in - r0, cc = 4 * s + col_in;
                    vals[slot] = (rr >= 0 && rr < N && cc <= rr) ? (float)Wc[rr * kLdsStride + cc]
                                                                  : 0.0f;
                    if (++slot == 4) {
                        Wq[gi * 64 + i] = make_float4(vals[0], vals[1], vals[2], vals[3]);
                        slot = 0;
                        ++gi;
                    }
                }
            }
            if (slot) {
                for (int z = slot; z < 4; ++z) vals[z] = 0.0f;
                Wq[gi * 64 + i] = make_float4(vals[0], vals[1], vals[2], vals[3]);
            }
            // signal as an FP32 pair in B-operand lane order: element g*16 + s
            // holds S_q[4s + g]
            float *Sp = reinterpret_cast<float *>(rq + wu);
            {
                const int g4 = i >> 4, s16 = i & 15, k = 4 * s16 + g4;
                const double sv = (k < N) ? Sq[k] : 0.0;
                const float hi = (float)sv;
                Sp[i] = hi;
                Sp[64 + i] = (float)(sv - (double)hi);
            }
            for (int u = wu + 32 + i; u < ru; u += 64) rq[u] = make_uint4(0u, 0u, 0u, 0u);
        }
        __syncthreads();
    }
}

hipError_t launch_cov_build(const fc_grid *g, const double *F, const double *stat, int stat_mode,
                            uint32_t forms, double *W64, uint4 *R32, unsigned long long *bad_q,
                            hipStream_t st)
{
    const int64_t blocks = g->G < 65536 ? g->G : 65536;
    hipLaunchKernelGGL(k_cov_build, dim3((unsigned)blocks), dim3(64), 0, st, g->S64, F, stat, g->N,
                       g->G, stat_mode, forms, g->ns, W64, R32, bad_q);
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
