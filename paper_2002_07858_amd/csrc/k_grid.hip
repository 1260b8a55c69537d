// k_grid.hip -- grid residency: the signal table in the scan's lane order.
//
// The FP32 scan forms each residual d - S(q) in FP64 and rounds it to FP32
// once, so its error is relative to the residual itself, not to the count
// level of S.  For that the scan reads S(q) in FP64, in the order in which
// lane group g needs bin 4s+g at k-step s.
#include "fc_internal.h"

namespace fcx {

// S64p[q][g*16 + s] = S[q][4s+g], zero past N.
__global__ __launch_bounds__(256) void k_stage_signal(const double *__restrict__ S64, int64_t G,
                                                     int N, double *__restrict__ S64p)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= G * 64) return;
    const int64_t q = e >> 6;
    const int w = (int)(e & 63);
    const int g = w >> 4, s = w & 15;
    const int k = 4 * s + g;
    S64p[e] = (k < N) ? S64[q * N + k] : 0.0;
}

hipError_t launch_stage_signal(const double *S64, int64_t G, int N, double *S64p, hipStream_t st)
{
    const int64_t n = G * 64;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_stage_signal, dim3((unsigned)blocks), dim3(256), 0, st, S64, G, N, S64p);
    return hipGetLastError();
}

}  // namespace fcx
