// k_crit.hip -- critical values and histogram of Delta chi^2 per true point.
//
// Section 1 / Figure 1: the critical value for a fraction alpha is the value
// left of which that fraction of the Delta chi^2 distribution lies.  It is
// taken as the type-1 order statistic x_(j), j = ceil(alpha K) clamped to
// [1, K], with NaN ordered last.  One block per segment finds x_(j) for every
// alpha at once by an 8-pass radix select (8 bits per pass) over 64-bit keys
// whose unsigned order is the numeric order of the doubles; no sort, no
// scratch memory beyond LDS counters.
#include "fc_internal.h"

namespace fcx {

constexpr int kMaxAlpha = 8;

struct AlphaArgs {
    double a[kMaxAlpha];
};

__device__ __forceinline__ unsigned long long order_key(double x)
{
    if (x != x) return ~0ull;  // NaN sorts last
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double from_order_key(unsigned long long k)
{
    if (k == ~0ull) return __builtin_nan("");
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// Segment s is x[seg_lo[s] .. seg_hi[s]).  The order statistics taken are
// ranks ceil(alpha K) (alpha mode), or ranks[s][a] (1-based, clamped to
// [1, K]) when a rank table is given.
__global__ __launch_bounds__(256) void k_crit(const int64_t *__restrict__ seg_lo,
                                             const int64_t *__restrict__ seg_hi,
                                             const double *__restrict__ x, int n_alpha,
                                             AlphaArgs alpha, const int64_t *__restrict__ ranks,
                                             double *__restrict__ crit, int n_bins,
                                             double hist_hi, int64_t *__restrict__ hist)
{
    __shared__ unsigned int cnt[kMaxAlpha][256];
    __shared__ unsigned long long prefix[kMaxAlpha];
    __shared__ long long rank[kMaxAlpha];
    extern __shared__ unsigned int hbin[];

    const int64_t sgi = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t lo = seg_lo[sgi], hi = seg_hi[sgi];
    const bool valid = lo >= 0 && hi >= lo;
    const int64_t K = valid ? hi - lo : 0;

    // ---- histogram ----------------------------------------------------------
    if (hist) {
        for (int b = tid; b <= n_bins; b += blockDim.x) hbin[b] = 0u;
        __syncthreads();
        const double width = hist_hi / (double)n_bins;
        for (int64_t k = tid; k < K; k += blockDim.x) {
            const double v = x[lo + k];
            int b = n_bins;
            if (v >= 0.0 && v < hist_hi) {
                const double f = floor(v / width);
                b = (f > (double)(n_bins - 1)) ? n_bins - 1 : (int)f;
            }
            atomicAdd(&hbin[b], 1u);
        }
        __syncthreads();
        for (int b = tid; b <= n_bins; b += blockDim.x)
            hist[sgi * (int64_t)(n_bins + 1) + b] = (int64_t)hbin[b];
    }

    // ---- radix select --------------------------------------------------------
    if (K == 0) {
        if (tid < n_alpha) crit[sgi * n_alpha + tid] = __builtin_nan("");
        return;
    }
    if (tid < n_alpha) {
        long long j = ranks ? (long long)ranks[sgi * n_alpha + tid]
                            : (long long)ceil(alpha.a[tid] * (double)K);
        if (j < 1) j = 1;
        if (j > K) j = K;
        rank[tid] = j - 1;  // 0-based
        prefix[tid] = 0ull;
    }
    __syncthreads();
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int e = tid; e < kMaxAlpha * 256; e += blockDim.x) (&cnt[0][0])[e] = 0u;
        __syncthreads();
        const unsigned long long himask = (shift == 56) ? 0ull : (~0ull << (shift + 8));
        for (int64_t k = tid; k < K; k += blockDim.x) {
            const unsigned long long key = order_key(x[lo + k]);
            const unsigned int digit = (unsigned int)((key >> shift) & 255ull);
            for (int a = 0; a < n_alpha; ++a)
                if ((key & himask) == prefix[a]) atomicAdd(&cnt[a][digit], 1u);
        }
        __syncthreads();
        // digit of rank r: one wave per fraction, lane l holding digits 4l..4l+3;
        // a prefix sum over the lanes finds the lane whose digits cover r
        const int wave = tid >> 6, lane = tid & 63;
        for (int a = wave; a < n_alpha; a += 4) {
            const long long r = rank[a];
            const long long c0 = cnt[a][4 * lane], c1 = cnt[a][4 * lane + 1],
                            c2 = cnt[a][4 * lane + 2], c3 = cnt[a][4 * lane + 3];
            const long long own = c0 + c1 + c2 + c3;
            long long incl = own;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const long long up = __shfl_up(incl, off, 64);
                if (lane >= off) incl += up;
            }
            const long long excl = incl - own;
            const long long total = __shfl(incl, 63, 64);
            if (excl <= r && r < incl) {
                long long rr = r - excl;
                unsigned int d = 4 * lane;
                if (rr >= c0) {
                    rr -= c0;
                    ++d;
                    if (rr >= c1) {
                        rr -= c1;
                        ++d;
                        if (rr >= c2) {
                            rr -= c2;
                            ++d;
                        }
                    }
                }
                rank[a] = rr;
                prefix[a] |= ((unsigned long long)d) << shift;
            } else if (lane == 63 && r >= total) {  // not reached for a consistent count
                rank[a] = r - total;
                prefix[a] |= 255ull << shift;
            }
        }
        __syncthreads();
    }
    if (tid < n_alpha) crit[sgi * n_alpha + tid] = from_order_key(prefix[tid]);
}

hipError_t launch_crit(int64_t n_seg, const int64_t *seg_off, const double *x, int n_alpha,
                       const double *alpha, double *crit, int n_bins, double hist_hi,
                       int64_t *hist, hipStream_t st)
{
    AlphaArgs aa;
    for (int a = 0; a < kMaxAlpha; ++a) aa.a[a] = (a < n_alpha) ? alpha[a] : 1.0;
    const size_t lds = hist ? sizeof(unsigned int) * (size_t)(n_bins + 1) : 0;
    hipLaunchKernelGGL(k_crit, dim3((unsigned)n_seg), dim3(256), lds, st, seg_off, seg_off + 1, x,
                       n_alpha, aa, nullptr, crit, n_bins, hist_hi, hist);
    return hipGetLastError();
}

hipError_t launch_crit_gapped(int64_t n_seg, const int64_t *seg_lo, const int64_t *seg_hi,
                              const double *x, int n_alpha, const double *alpha, double *crit,
                              hipStream_t st)
{
    AlphaArgs aa;
    for (int a = 0; a < kMaxAlpha; ++a) aa.a[a] = (a < n_alpha) ? alpha[a] : 1.0;
    hipLaunchKernelGGL(k_crit, dim3((unsigned)n_seg), dim3(256), 0, st, seg_lo, seg_hi, x, n_alpha,
                       aa, nullptr, crit, 0, 1.0, nullptr);
    return hipGetLastError();
}

hipError_t launch_select_ranks(int64_t n_seg, const int64_t *seg_lo, const int64_t *seg_hi,
                               const double *x, int n_q, const int64_t *ranks, double *out,
                               hipStream_t st)
{
    AlphaArgs aa;
    for (int a = 0; a < kMaxAlpha; ++a) aa.a[a] = 1.0;
    hipLaunchKernelGGL(k_crit, dim3((unsigned)n_seg), dim3(256), 0, st, seg_lo, seg_hi, x, n_q, aa,
                       ranks, out, 0, 1.0, nullptr);
    return hipGetLastError();
}

}  // namespace fcx
