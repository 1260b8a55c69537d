// k_grid.hip -- per-bin offset of the signal grid for the split forms.
//
// The split forms evaluate z = W_q (d - o) - W_q (S_q - o) with a per-bin
// offset o, the mean of S over the grid, and scale (d - o) by a power of two
// chosen from max_q |S_q - o| (FP16 range).  One block per bin; a fixed
// strided split and a fixed LDS tree keep both reductions deterministic.
#include "fc_internal.h"

namespace fcx {

__global__ __launch_bounds__(256) void k_offset(const double *__restrict__ S64, int64_t G, int N,
                                               double *__restrict__ off, double *__restrict__ dev)
{
    __shared__ double part[256];
    const int j = blockIdx.x;
    const int t = threadIdx.x;
    double acc = 0.0;
    if (j < N)
        for (int64_t q = t; q < G; q += blockDim.x) acc += S64[q * N + j];
    part[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    const double o = (j < N) ? part[0] / (double)G : 0.0;
    __syncthreads();
    double mx = 0.0;
    if (j < N)
        for (int64_t q = t; q < G; q += blockDim.x) mx = fmax(mx, fabs(S64[q * N + j] - o));
    part[t] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] = fmax(part[t], part[t + w]);
        __syncthreads();
    }
    if (t == 0) {
        off[j] = o;
        dev[j] = part[0];
    }
}

hipError_t launch_offset(const double *S64, int64_t G, int N, double *off, double *dev,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_offset, dim3(kMaxBins), dim3(256), 0, st, S64, G, N, off, dev);
    return hipGetLastError();
}

}  // namespace fcx
