// k_gen.hip -- universes drawn on the device.
//
// Section 2, steps 1-2 of the per-universe procedure: the prediction S(p) at
// the true point is fluctuated into a fake data vector d.  Here d is Poisson
// counts around S(p) plus a correlated Gaussian fractional systematic,
//     d_i = n_i + S_p[i] * (L_F g)_i,   n_i ~ Poisson(S_p[i]),  g ~ N(0, I),
// with L_F the Cholesky factor of the fractional covariance F, so that
// Cov(d) = diag(S_p) + F o (S_p S_p^T), the covariance the scan assumes.
//
// Every random number comes from a counter-based stream, so a universe
// depends only on (seed, p, j) and any batching of the work gives the same
// values:
//   Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11), key (seed, 0);
//   block b of purpose t (0 Poisson, 1 normal) for point p, universe j, bin i
//   has counter (j, p, i << 32 | t << 28 | b, 0);
//   a 64-bit word w is the uniform ((w >> 11) + 0.5) 2^-53 in (0, 1).
// Poisson(lambda): 0 for lambda = 0; the multiplication method below 10 (the
// product of successive uniforms, first at or below exp(-lambda), at most
// 1024 of them); Hormann's transformed rejection with squeeze (PTRS, 1993)
// from 10 up (attempt t uses words 2(t%2), 2(t%2)+1 of block t/2, at most 512
// attempts, then floor(lambda)).  Normal: Box-Muller, sqrt(-2 ln u0)
// cos(2 pi u1) from words 0 and 1 of the bin's normal block.  A mean that is
// negative, NaN or infinite gives count -1 and d = NaN.
//
// One wave per universe, lane i = bin i; L_F sits in LDS.  The arithmetic is
// FP64 without contraction, in the order written, so the counts are the same
// integers on any IEEE machine that evaluates exp/log/lgamma to within an ulp
// (a decision flips only if a uniform lands within rounding of a boundary).
#include "fc_internal.h"

namespace fcx {

#pragma clang fp contract(off)

__device__ __forceinline__ void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
        const uint64_t hi0 = __umul64hi(m0, x[0]), lo0 = m0 * x[0];
        const uint64_t hi1 = __umul64hi(m1, x[2]), lo1 = m1 * x[2];
        const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

__device__ __forceinline__ void stream_block(uint64_t seed, int64_t p, int64_t j, int i,
                                             uint32_t purpose, uint32_t b, uint64_t w[4])
{
    w[0] = (uint64_t)j;
    w[1] = (uint64_t)p;
    w[2] = ((uint64_t)(uint32_t)i << 32) | ((uint64_t)purpose << 28) | (uint64_t)b;
    w[3] = 0;
    philox4x64_10(w, seed, 0);
}

__device__ __forceinline__ double unit_open(uint64_t w)
{
    return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

// Poisson count for bin i of universe j at point p (-1: no valid mean).
__device__ int64_t poisson_draw(double lam, uint64_t seed, int64_t p, int64_t j, int i)
{
    if (!(lam >= 0.0) || __builtin_isinf(lam)) return -1;
    if (lam == 0.0) return 0;
    uint64_t w[4];
    if (lam < 10.0) {
        const double floor_p = exp(-lam);
        double prod = 1.0;
        int64_t k = 0;
        for (uint32_t b = 0; b < 256; ++b) {
            stream_block(seed, p, j, i, 0, b, w);
            for (int e = 0; e < 4; ++e) {
                prod = prod * unit_open(w[e]);
                if (prod <= floor_p) return k;
                k = k + 1;
            }
        }
        return k;
    }
    // PTRS constants (functions of sqrt(lambda) only)
    const double sq = sqrt(lam), ll = log(lam);
    const double B = 0.931 + 2.53 * sq;
    const double A = -0.059 + 0.02483 * B;
    const double ia = 1.1239 + 1.1328 / (B - 3.4);
    const double vr = 0.9277 - 3.6224 / (B - 2.0);
    for (uint32_t t = 0; t < 512; ++t) {
        if ((t & 1u) == 0u) stream_block(seed, p, j, i, 0, t >> 1, w);
        const int h = 2 * (int)(t & 1u);
        const double U = unit_open(w[h]) - 0.5;
        const double V = unit_open(w[h + 1]);
        const double us = 0.5 - fabs(U);
        const double kf = floor((2.0 * A / us + B) * U + lam + 0.43);
        if (us >= 0.07 && V <= vr) return (int64_t)kf;         // squeeze: accept
        if (kf < 0.0 || (us < 0.013 && V > us)) continue;      // outside the hat
        const double lhs = log(V * ia / (A / (us * us) + B));
        const double rhs = -lam + kf * ll - lgamma(kf + 1.0);
        if (lhs <= rhs) return (int64_t)kf;
    }
    return (int64_t)floor(lam);
}

__device__ __forceinline__ double normal_draw(uint64_t seed, int64_t p, int64_t j, int i)
{
    uint64_t w[4];
    stream_block(seed, p, j, i, 1, 0, w);
    const double u0 = unit_open(w[0]), u1 = unit_open(w[1]);
    return sqrt(-2.0 * log(u0)) * cos(6.283185307179586 * u1);
}

// Cholesky factor of the fractional covariance, one 64-lane block, lane i
// owning row i (right-looking, in LDS).  flag = 1 if positive definite.
__global__ __launch_bounds__(64) void k_chol_frac(const double *__restrict__ F, int N,
                                                  double *__restrict__ LF, int *__restrict__ flag)
{
    __shared__ double A[kMaxBins * kMaxBins];
    const int i = threadIdx.x;
    for (int e = i; e < N * N; e += 64) A[e] = F[e];
    __syncthreads();
    bool ok = true;
    for (int c = 0; c < N; ++c) {
        const double piv = A[c * N + c];
        if (!(piv > 0.0)) {  // every lane read the same pivot
            ok = false;
            break;
        }
        const double lcc = sqrt(piv);
        __syncthreads();
        if (i == c) A[c * N + c] = lcc;
        if (i > c && i < N) A[i * N + c] = A[i * N + c] / lcc;
        __syncthreads();
        if (i > c && i < N) {
            const double lic = A[i * N + c];
            for (int k = c + 1; k <= i; ++k) A[i * N + k] = A[i * N + k] - lic * A[k * N + c];
        }
        __syncthreads();
    }
    if (i < N)
        for (int k = 0; k < N; ++k) LF[i * N + k] = (ok && k <= i) ? A[i * N + k] : 0.0;
    if (i == 0) *flag = ok ? 1 : 0;
}

// Largest k in [0, n) with seg_off[k] <= r (seg_off non-decreasing).
__device__ __forceinline__ int64_t segment_of(const int64_t *__restrict__ seg_off, int64_t n,
                                              int64_t r)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (seg_off[mid] <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_gen_universes(
    const double *__restrict__ S64, const double *__restrict__ LF, int N, int64_t G,
    int64_t n_pts, const int64_t *__restrict__ p, const int64_t *__restrict__ seg_off,
    const int64_t *__restrict__ u_first, uint64_t seed, int64_t K, double *__restrict__ d,
    int64_t *__restrict__ p_idx, int32_t *__restrict__ counts)
{
    __shared__ double lf[kMaxBins * kMaxBins];
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) lf[e] = LF[e];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t r = wave; r < K; r += n_waves) {
        const int64_t k = segment_of(seg_off, n_pts, r);
        const int64_t pk = p[k];
        const int64_t j = (u_first ? u_first[k] : 0) + (r - seg_off[k]);
        const bool valid = pk >= 0 && pk < G;
        double g = 0.0, lam = 0.0;
        int64_t n = -1;
        if (valid && lane < N) {
            lam = S64[pk * N + lane];
            g = normal_draw(seed, pk, j, lane);
            n = poisson_draw(lam, seed, pk, j, lane);
        }
        // z_i = sum_{l <= i} L_F[i][l] g_l, increasing l
        double z = 0.0;
        for (int l = 0; l < N; ++l) {
            const double gl = __shfl(g, l);
            if (l <= lane) z = z + lf[(lane < N ? lane : 0) * N + l] * gl;
        }
        if (lane < N) {
            d[r * N + lane] = (n < 0) ? __builtin_nan("") : (double)n + lam * z;
            if (counts) counts[r * N + lane] = (int32_t)n;
        }
        if (lane == 0 && p_idx) p_idx[r] = valid ? pk : -1;
    }
}

hipError_t launch_chol_frac(const double *F, int N, double *LF, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_chol_frac, dim3(1), dim3(64), 0, st, F, N, LF, flag);
    return hipGetLastError();
}

hipError_t launch_gen_universes(const fc_grid *g, int64_t n_pts, const int64_t *p,
                                const int64_t *seg_off, const int64_t *u_first, uint64_t seed,
                                int64_t K, double *d, int64_t *p_idx, int32_t *counts,
                                hipStream_t st)
{
    const int64_t rows_per_block = 4;
    int64_t blocks = (K + rows_per_block - 1) / rows_per_block;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_gen_universes, dim3((unsigned)blocks), dim3(256), 0, st, g->S64, g->LF64,
                       g->N, g->G, n_pts, p, seg_off, u_first, seed, K, d, p_idx, counts);
    return hipGetLastError();
}

}  // namespace fcx
