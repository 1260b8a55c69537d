// k_data.hip -- the observed-data statistic and the FC acceptance region.
//
// Section 1: the scan's purpose is to find the grid points compatible with
// the central (observed) data vector c.  With the per-point critical values
// of the Delta chi^2 distribution (built from the universes of each true
// point), a point p is accepted when the data's own statistic
//     Delta chi2_data(p) = chi2(c, S(p)) - min_q chi2(c, S(q))
// is not above its critical value.  chi2(c, q) is evaluated for every q in
// FP64 with the FP64 factor (one wave per grid point, lane i owning row i of
// W_q), the minimum with Algorithm 1's rule (lowest q among exact ties).
#include "fc_internal.h"

namespace fcx {

__device__ __forceinline__ unsigned long long dorder(double x)
{
    if (x != x) return ~0ull;
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(64) void k_data_chi2(const double *__restrict__ W64,
                                                 const double *__restrict__ S64,
                                                 const double *__restrict__ c, int N, int64_t G,
                                                 double *__restrict__ chi2,
                                                 unsigned long long *__restrict__ min_key)
{
    const int i = threadIdx.x;
    const int64_t NT = (int64_t)N * (N + 1) / 2;
    for (int64_t q = blockIdx.x; q < G; q += gridDim.x) {
        const double *Wq = W64 + q * NT;
        const double *Sq = S64 + q * N;
        double z = 0.0;
        if (i < N) {
            const double *row = Wq + (int64_t)i * (i + 1) / 2;
            for (int j = 0; j <= i; ++j) z = fma(row[j], c[j] - Sq[j], z);
        }
        double v = z * z;
        for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
        if (i == 0) {
            chi2[q] = v;
            atomicMin(min_key, dorder(v));
        }
    }
}

// Lowest q whose chi2 equals the minimum; then Delta chi2_data = chi2 - min.
__global__ __launch_bounds__(256) void k_data_argmin(const double *__restrict__ chi2, int64_t G,
                                                    const unsigned long long *__restrict__ min_key,
                                                    unsigned long long *__restrict__ arg)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= G) return;
    if (dorder(chi2[q]) == *min_key) atomicMin(arg, (unsigned long long)q);
}

__device__ __forceinline__ double dorder_inv(unsigned long long k)
{
    if (k == ~0ull) return __builtin_nan("");
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// In place: every thread reads only its own element, and the minimum comes
// from its key, so no block depends on another's writes.
__global__ __launch_bounds__(256) void k_data_delta(double *__restrict__ chi2, int64_t G,
                                                   const unsigned long long *__restrict__ min_key)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= G) return;
    chi2[q] = chi2[q] - dorder_inv(*min_key);  // all-NaN data: no minimum, NaN
}

__global__ __launch_bounds__(256) void k_accept(int64_t n_pts, const int64_t *__restrict__ p,
                                               const double *__restrict__ crit, int64_t stride,
                                               const double *__restrict__ dchi2_data, int64_t G,
                                               uint8_t *__restrict__ accepted)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_pts) return;
    const int64_t q = p[k];
    uint8_t a = 0;
    if (q >= 0 && q < G) a = (dchi2_data[q] <= crit[k * stride]) ? 1 : 0;
    accepted[k] = a;
}

hipError_t launch_data_scan(const fc_grid *g, const double *c, double *chi2,
                            unsigned long long *scratch /* [2] */, hipStream_t st)
{
    const unsigned long long init[2] = {~0ull, ~0ull};
    hipError_t e = hipMemcpyAsync(scratch, init, sizeof(init), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    const int64_t blocks = g->G < 65536 ? g->G : 65536;
    hipLaunchKernelGGL(k_data_chi2, dim3((unsigned)blocks), dim3(64), 0, st, g->W64, g->S64, c,
                       g->N, g->G, chi2, scratch);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t b2 = (g->G + 255) / 256;
    hipLaunchKernelGGL(k_data_argmin, dim3((unsigned)b2), dim3(256), 0, st, chi2, g->G, scratch,
                       scratch + 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_data_delta, dim3((unsigned)b2), dim3(256), 0, st, chi2, g->G, scratch);
    return hipGetLastError();
}

hipError_t launch_accept(int64_t n_pts, const int64_t *p, const double *crit, int64_t stride,
                         const double *dchi2_data, int64_t G, uint8_t *accepted, hipStream_t st)
{
    const int64_t blocks = (n_pts + 255) / 256;
    hipLaunchKernelGGL(k_accept, dim3((unsigned)blocks), dim3(256), 0, st, n_pts, p, crit, stride,
                       dchi2_data, G, accepted);
    return hipGetLastError();
}

}  // namespace fcx
