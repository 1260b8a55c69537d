// fc_internal.h -- private declarations shared by the library's host code and
// kernels.  Not part of the C ABI (include/fc.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "fc.h"

// ---------------------------------------------------------------------------
// FP32 factor layout for the MFMA scan.
//
// The scan computes z = W_q r for a tile of universes with
// v_mfma_f32_16x16x4_f32: A = a 16x4 block of W_q (rows = z index, cols =
// bins), B = a 4x16 block of R (bins x universes).  Bins are taken four at a
// time ("k-steps", ns = ceil(N/4)); z rows sixteen at a time ("row blocks",
// nb = ceil(N/16)).  W_q is lower triangular, so row block b only needs the
// k-steps s <= 4b+3.  The (s, b) pairs actually needed are enumerated with s
// outer and b = s/4 .. nb-1 inner; pair t holds, for lane l, the value
// W_q[16b + l%16][4s + l/16] (the A-operand layout).  Per grid point the pairs
// are stored lane-major in groups of four:
//     W32[q][t/4][lane][t%4]           (ng = ceil(npair/4) groups)
// so that every lane fetches its next four A values with one 16-byte load and
// a wave reads 1 KB contiguously.
//
// The signal is kept in FP64 and also stored per grid point in the lane order
// of the B operand,
//     S64p[q][g][s] = S_q[4s+g]   (g = 0..3, s = 0..15, zero past N)
// so that the residual d - S_q is formed in FP64 and rounded to FP32 once.
// ---------------------------------------------------------------------------
namespace fcx {

constexpr int kMaxBins = FC_MAX_BINS;
constexpr int kWavesPerBlock = 4;
constexpr int kScanColBlocks = 2;  // 16-universe column blocks per wave (32 universes)

__host__ __device__ constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ constexpr int n_ksteps(int N) { return ceil_div(N, 4); }
__host__ __device__ constexpr int n_rowblocks_from_ns(int ns) { return ceil_div(ns, 4); }
__host__ __device__ constexpr int n_pairs_from_ns(int ns) {
    int nb = n_rowblocks_from_ns(ns), t = 0;
    for (int s = 0; s < ns; ++s) t += nb - s / 4;
    return t;
}
__host__ __device__ constexpr int n_groups_from_ns(int ns) { return ceil_div(n_pairs_from_ns(ns), 4); }

// Packed lower-triangle index for the FP64 factor.
__host__ __device__ inline int64_t tri_index(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }

// Key of the running minimum: FP32 chi^2 bits (non-negative, so ordered as
// unsigned) above the grid index; the integer minimum over keys is the
// smallest chi^2 with ties broken by the lowest q.
constexpr uint64_t kKeyNone = (uint64_t(0x7f800000u) << 32) | 0xffffffffu;

}  // namespace fcx

struct fc_grid {
    int device = 0;
    int32_t D = 0, N = 0;
    int64_t G = 0;
    std::vector<int64_t> axis_len;
    std::vector<double> axis_vals;
    std::vector<double> central;
    double *S64 = nullptr;   // device [G][N]
    double *S64p = nullptr;  // device [G][64], see layout above
    uint32_t forms = 0;
    double *W64 = nullptr;  // device [G][N(N+1)/2], packed lower W_q = L_q^{-1}
    float *W32 = nullptr;   // device [G][ng][64][4]
    size_t bytes = 0;
    int ns = 0, ng = 0;     // FP32 fragment geometry
};

// ---- launchers (defined in the .hip files) ------------------------------
namespace fcx {

hipError_t launch_stage_signal(const double *S64, int64_t G, int N, double *S64p, hipStream_t st);
hipError_t launch_cov_build(const fc_grid *g, const double *F, const double *stat, int stat_mode,
                            uint32_t forms, double *W64, float *W32, unsigned long long *bad_q,
                            hipStream_t st);
hipError_t launch_scan_fp32(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                            unsigned long long *keys, double *chi2_p, hipStream_t st);
hipError_t launch_scan_fp64(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                            double *dchi2, double *chi2_min, int64_t *argmin, double *chi2_p,
                            hipStream_t st);
hipError_t launch_init_keys(int64_t K, unsigned long long *keys, double *chi2_p, hipStream_t st);
hipError_t launch_finalize(int64_t K, const int64_t *p_idx, unsigned long long *keys_as_chi2_min,
                           int64_t *argmin, const double *chi2_p, double *dchi2, hipStream_t st);
hipError_t launch_inverse_cov(const fc_grid *g, int64_t q0, int64_t nq, double *out,
                              hipStream_t st);
hipError_t launch_crit(int64_t n_seg, const int64_t *seg_off, const double *x, int n_alpha,
                       const double *alpha, double *crit, int n_bins, double hist_hi,
                       int64_t *hist, hipStream_t st);

// Scan launch geometry chosen by the host: universe tiles x grid chunks.
struct ScanGeometry {
    int64_t n_utiles = 0;
    int64_t n_qchunks = 0;
    int64_t q_per_chunk = 0;
};
ScanGeometry scan_geometry(int64_t K, int64_t G, int slots, int univ_per_block);

}  // namespace fcx
