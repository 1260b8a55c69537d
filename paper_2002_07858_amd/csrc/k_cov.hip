// k_cov.hip -- launch of the covariance build (k_cov_impl.h: the per-point
// FP64 Cholesky and inverse factor, one kernel per padded bin count, compiled
// in the k_cov_np_*.hip files) and Sigma_q^{-1} = W_q^T W_q for inspection.
#include <stdint.h>

#include "fc_internal.h"

namespace fcx {

template <int NP>
hipError_t launch_cov_np(const fc_grid *g, const double *F, const double *stat, int stat_mode,
                         uint32_t forms, const int16_t *maps, double *W64, uint4 *R64, uint4 *R32,
                         uint4 *RB16, uint4 *RH16, unsigned long long *bad_q, hipStream_t st);

hipError_t launch_cov_build(const fc_grid *g, const double *F, const double *stat, int stat_mode,
                            uint32_t forms, const int16_t *maps, double *W64, uint4 *R64,
                            uint4 *R32, uint4 *RB16, uint4 *RH16, unsigned long long *bad_q,
                            hipStream_t st)
{
    switch ((g->N + 3) / 4) {
#define FC_NP(n)                                                                               \
    case n:                                                                                    \
        return launch_cov_np<4 * n>(g, F, stat, stat_mode, forms, maps, W64, R64, R32, RB16, \
                                    RH16, bad_q, st);
        FC_NP(1) FC_NP(2) FC_NP(3) FC_NP(4) FC_NP(5) FC_NP(6) FC_NP(7) FC_NP(8)
        FC_NP(9) FC_NP(10) FC_NP(11) FC_NP(12) FC_NP(13) FC_NP(14) FC_NP(15) FC_NP(16)
#undef FC_NP
    }
    return hipErrorInvalidValue;
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
