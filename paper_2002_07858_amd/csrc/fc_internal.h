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
// The scan computes z = W_q r with v_mfma_f32_4x4x1_16b_f32, one universe per
// lane: B is the lane's own residual at one bin, so lane l of output
// register j accumulates row 4b + j of W_q r for universe l, and chi^2 is the
// lane's own sum of squares (no cross-lane reduction).  The A operand of each
// instruction is one 4-row, 1-bin slice of W_q, broadcast from one of the 16
// four-lane blocks of an A register (CBSZ = 4, ABID = slot), so one register
// carries 16 slices.  Rows and bins are padded at the top/left by
// P = 4 ns - N (ns = ceil(N/4)): padded index x' = x + P, so that the short
// row block is the narrowest one.  Row block b (padded rows 4b .. 4b+3) needs
// padded bins k' <= 4b + 3.  The (k', b) pairs are enumerated k' outer
// (0 .. 4ns-1), b inner (k'/4 .. ns-1): npair = 2 ns (ns+1); the P ns pairs
// with k' < P are zero and skipped by the scan (N = 57: 435 of 480).  Pair t
// lives in A register t/16, slot t%16; lane 4 (t%16) + m holds
//     W_q[4b + m - P][k' - P]                    (zero outside the triangle)
// Per grid point the A registers are stored lane-major in groups of four,
//     A[v/4][lane][v%4]               (ng = ceil(npair/64) groups of 1 KB)
// so that a lane fetches four registers with one 16-byte access and a wave
// reads 1 KB contiguously.  They are followed by the signal's FP32 part (real
// bin order, read through the scalar cache) and by the W-image of its rounding
// error (padded row order, the accumulators' start),
//     Sh[k]  = float(S_q[k])                                      (k < 64)
//     C[r']  = float(-sum_k W_q[r' - P][k] (S_q[k] - float(S_q[k])))  (r' < 64)
// (zero outside the real bins / rows; 256 B each).  With d = dh + dl split the
// same way, W_q (d - S_q) = W_q ((dh - Sh) + dl) + C up to rounding, so the
// residual costs two FP32 instructions, its error is relative to the residual
// itself, and C is the accumulators' initial value.  One grid point's record
// is rec_units(ns) 16-byte units, unpadded; the scan's 256 threads copy it
// with direct global -> LDS loads, the last piece predicated.
// ---------------------------------------------------------------------------
namespace fcx {

constexpr int kMaxBins = FC_MAX_BINS;
constexpr int kWavesPerBlock = 4;
constexpr int kFp32UnivPerBlock = 64 * kWavesPerBlock;  // one universe per lane
constexpr int kPtsWaves = 4;                 // waves per block of the points scan
constexpr int kPtsTile = 64 * kPtsWaves;     // its universes per tile

__host__ __device__ constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ constexpr int n_ksteps(int N) { return ceil_div(N, 4); }
__host__ __device__ constexpr int fp32_pad(int ns, int N) { return 4 * ns - N; }
__host__ __device__ constexpr int fp32_npairs(int ns) { return 2 * ns * (ns + 1); }
__host__ __device__ constexpr int n_groups_from_ns(int ns) { return ceil_div(fp32_npairs(ns), 64); }
__host__ __device__ constexpr int rec_w_units(int ns) { return n_groups_from_ns(ns) * 64; }
__host__ __device__ constexpr int rec_units(int ns) { return rec_w_units(ns) + 32; }
// Index of pair (k', b) in the enumeration order (k' outer, b inner).
__host__ __device__ constexpr int fp32_pair_index(int ns, int kp, int b)
{
    int t = 0;
    for (int c = 0; c < kp; ++c) t += ns - c / 4;
    return t + (b - kp / 4);
}
// Padded bin k' and row block b of pair t (t < npair).
__host__ __device__ constexpr int fp32_pair_kp(int ns, int t)
{
    int kp = 0;
    while (t >= ns - kp / 4) {
        t -= ns - kp / 4;
        ++kp;
    }
    return kp;
}
__host__ __device__ constexpr int fp32_pair_b(int ns, int t)
{
    const int kp = fp32_pair_kp(ns, t);
    return kp / 4 + (t - fp32_pair_index(ns, kp, kp / 4));
}

// ---------------------------------------------------------------------------
// Split-form layout (hi+lo BF16 or FP16 operands, FP32 accumulation) for
// v_mfma_f32_16x16x32_{bf16,f16}: A = 16x32 fragments of the factor, B = 32x16
// fragments of the universes.  The split forms use linearity,
//     z = W_q (d - S_q) = W_q (d - o) - W_q (S_q - o),
// so that the universes are split once (registers, for the whole scan) and
// u_q = W_q (S_q - o) is computed per grid point in FP64 when the form is
// built; o is a per-bin offset (the grid mean of S).
//
// The three products hi*hi + hi*lo + lo*hi of a bin sit next to each other
// along k: position p = 3 j + t holds bin j, with (A, B) = (W_hi, d_hi) for
// t = 0, (W_hi, d_lo) for t = 1 and (W_lo, d_hi) for t = 2, so a row needing
// bins 0..r needs the first 3 (r + 1) positions and no product is padded to
// a 32-position step on its own.  Rows go in nb = ceil(N/16) groups of at
// most 16, every group but the first full (group g holds rows
// row0(g) .. row0(g+1)-1, row0(0) = 0, row0(g) = N - 16 (nb - g)), which
// keeps each group's last row, and so its step count
// steps(g) = ceil(3 row0(g+1) / 32), as small as 16-row groups allow (N = 57:
// rows 0-8 | 9-24 | 25-40 | 41-56, 1 + 3 + 4 + 6 = 14 steps of 32 positions,
// where a separate 32-bin padding of each product takes 18).
//
// Fragment f = (g, s), numbered group by group, holds in lane l the eight A
// values at positions 32 s + 8 (l/16) + e, e = 0..7, of row row0(g) + l%16
// (zero past the group's last row or the row's last bin), W_q scaled by 2^eq
// (FP16 form).  Record of one grid point (16 B units):
//     [fragment][lane]                                  nfrag * 64 units
//     c[l/16][g][j] FP32, -2^(eq+ed) u_q[row0(g) + 4 (l/16) + j]   16 units
//     {2^-2(eq+ed), 0, 0, 0}                                        1 unit
// c is the initial accumulator of every row group (zero on padding rows), so
// that the MFMA chain ends at 2^(eq+ed) z and chi^2 = 2^-2(eq+ed) sum z'^2.
// eq is chosen per grid point so that max |W_q| 2^eq lies in [2^13, 2^14); ed
// per grid so that max |S - o| 2^ed is below 2^13 (both 0 for BF16, whose
// range is FP32's).  The step counts of the groups, four bits each, name the
// kernel that scans the form (`split_code`).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int split_nb(int N) { return ceil_div(N, 16); }
__host__ __device__ constexpr int split_row0(int N, int g)
{
    return g <= 0 ? 0 : (g >= split_nb(N) ? N : N - 16 * (split_nb(N) - g));
}
__host__ __device__ constexpr int split_steps(int N, int g)
{
    return g < split_nb(N) ? ceil_div(3 * split_row0(N, g + 1), 32) : 0;
}
__host__ __device__ constexpr int split_code(int N)
{
    return split_steps(N, 0) | split_steps(N, 1) << 4 | split_steps(N, 2) << 8 |
           split_steps(N, 3) << 12;
}
// the same figures from a code
__host__ __device__ constexpr int code_steps(int code, int g) { return (code >> (4 * g)) & 15; }
__host__ __device__ constexpr int code_nb(int code)
{
    return (code_steps(code, 0) != 0) + (code_steps(code, 1) != 0) + (code_steps(code, 2) != 0) +
           (code_steps(code, 3) != 0);
}
__host__ __device__ constexpr int code_smax(int code)
{
    int m = 0;
    for (int g = 0; g < 4; ++g) m = code_steps(code, g) > m ? code_steps(code, g) : m;
    return m;
}
__host__ __device__ constexpr int code_nfrag(int code)
{
    return code_steps(code, 0) + code_steps(code, 1) + code_steps(code, 2) + code_steps(code, 3);
}
__host__ __device__ constexpr int code_frag(int code, int g, int s)
{
    int t = s;
    for (int g2 = 0; g2 < g; ++g2) t += code_steps(code, g2);
    return t;
}
// The i-th fragment in the scan's issue order (steps outer, groups inner):
// its step and its group.
__host__ __device__ constexpr int code_issue_s(int code, int i)
{
    for (int s = 0; s < 16; ++s)
        for (int g = 0; g < 4; ++g)
            if (s < code_steps(code, g) && i-- == 0) return s;
    return -1;
}
__host__ __device__ constexpr int code_issue_g(int code, int i)
{
    for (int s = 0; s < 16; ++s)
        for (int g = 0; g < 4; ++g)
            if (s < code_steps(code, g) && i-- == 0) return g;
    return -1;
}
__host__ __device__ constexpr int code_u_unit(int code) { return code_nfrag(code) * 64; }
__host__ __device__ constexpr int code_scale_unit(int code) { return code_u_unit(code) + 16; }
__host__ __device__ constexpr int code_rec_units(int code) { return code_scale_unit(code) + 1; }
__host__ __device__ constexpr int split_rec_units(int N) { return code_rec_units(split_code(N)); }

// ---------------------------------------------------------------------------
// FP64 tile form for v_mfma_f64_4x4x4f64 (four 4x4x4 blocks; the tile of W is
// the A operand of every block).  Bins and rows are padded to NP = 4 nb with
// nb = ceil(N / 4) blocks of four, real bins / rows at padded positions
// P .. NP-1 (P = NP - N): W'[r'][k'] = W_q[r' - P][k' - P] for P <= k' <= r',
// else 0.  The first bin block holds only L = 4 - P real bins; when L <= 2
// (N = 57: one) its products are cheaper on the vector ALUs than as nb tiles
// that are mostly zero, so the record carries those L columns apart ("lead"
// columns) and the tiles start at bin block k0 = 1; otherwise k0 = 0.  Tiles
// (kb, r) with k0 <= kb <= r (rows 4r .. 4r+3, bins 4kb .. 4kb+3) run kb outer,
// r inner.  Tile t's element A[i][k] = W'[4r + i][4kb + k] is stored at
// position 4k + i of the tile; tiles are stored in pairs,
// [pair][position][tile 2 pair + {0, 1}] doubles (an odd last pair padded
// with zeros), so that one 16-byte LDS read at pair * 256 +
// (4 (lane / 16) + lane % 4) * 16 gives a lane the A operands of two
// consecutive tiles.  Then, in the order a lane reads them (g = lane / 16,
// nbe = nb rounded up to even, 16-byte loads):
//     signal  Sp[g][r]    = S_q[4r + g - P]           (0 for padding)
//     lead    Wl[c][g][r] = W'[4r + g][P + c]  c < L  (lead columns only)
// N = 57: nb = 15, 105 tiles + 1 lead column, 14.3 KB per grid point.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int f64_nb(int N) { return (N + 3) / 4; }
__host__ __device__ constexpr int f64_pad(int N) { return 4 * f64_nb(N) - N; }
__host__ __device__ constexpr int f64_lead(int N)
{
    return (4 - f64_pad(N) <= 2) ? 4 - f64_pad(N) : 0;
}
__host__ __device__ constexpr int f64_k0(int N) { return f64_lead(N) ? 1 : 0; }
__host__ __device__ constexpr int f64_nbe(int N) { return (f64_nb(N) + 1) & ~1; }
__host__ __device__ constexpr int f64_ntile(int N)
{
    return (f64_nb(N) - f64_k0(N)) * (f64_nb(N) - f64_k0(N) + 1) / 2;
}
__host__ __device__ constexpr int f64_npair(int N) { return (f64_ntile(N) + 1) / 2; }
__host__ __device__ constexpr int f64_sig_double(int N) { return 32 * f64_npair(N); }
__host__ __device__ constexpr int f64_lead_double(int N)
{
    return f64_sig_double(N) + 4 * f64_nbe(N);
}
__host__ __device__ constexpr int f64_rec_doubles(int N)
{
    return f64_lead_double(N) + 4 * f64_nbe(N) * f64_lead(N);
}
__host__ __device__ constexpr int f64_rec_units(int N) { return f64_rec_doubles(N) / 2; }
__host__ __device__ constexpr int f64_tile_kb(int N, int t)
{
    int kb = f64_k0(N);
    while (t >= f64_nb(N) - kb) {
        t -= f64_nb(N) - kb;
        ++kb;
    }
    return kb;
}
__host__ __device__ constexpr int f64_tile_r(int N, int t)
{
    int kb = f64_k0(N);
    while (t >= f64_nb(N) - kb) {
        t -= f64_nb(N) - kb;
        ++kb;
    }
    return kb + t;
}

// (minimum, first grid point reaching it) of one grid chunk of the FP64 scan.
struct Fp64Part {
    double v;
    int64_t q;
};

// Copy one record of REC 16-byte units into LDS with direct global -> LDS
// loads: thread tid moves units tid, tid + 256, ...; each wave's 64 lanes land
// contiguously at its own base, so the LDS image equals the global record.  The loads are
// waited for (vmcnt) before the barrier that hands the buffer over.
#ifdef __HIPCC__
template <int REC, int THREADS>
__device__ __forceinline__ void record_to_lds(const uint4 *__restrict__ rec, uint4 *dst, int tid)
{
    // wave-uniform LDS base (M0) and a 32-bit lane offset on a uniform record base;
    // lanes past the record's last unit load nothing
    constexpr int CPT = (REC + THREADS - 1) / THREADS;
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
    const unsigned lane_off = (unsigned)tid * 16u;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
        if ((REC % THREADS) == 0 || c + 1 < CPT || c * THREADS + tid < REC)
            __builtin_amdgcn_global_load_lds(
                (const void *)(reinterpret_cast<const char *>(rec + c * THREADS) + lane_off),
                (__attribute__((address_space(3))) void *)(dst + c * THREADS + wbase), 16, 0, 0);
}

__device__ __forceinline__ void wait_record_loads()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt not waited for
}
#endif

// Packed lower-triangle index for the FP64 factor.
__host__ __device__ inline int64_t tri_index(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }

// ---------------------------------------------------------------------------
// Gather maps of the covariance build's record writers.  After the
// factorisation the build holds W_q in LDS as packed rows (W_q[r][c] at
// r (r + 1) / 2 + c) and S_q beside it; every record element is then one
// gather, whose source depends only on N (and ns) and is tabulated once per
// build: kMapZero -> 0, below kMapSig -> the packed W_q index, from kMapSig ->
// S_q[m - kMapSig].
// ---------------------------------------------------------------------------
constexpr int16_t kMapZero = -1;
constexpr int16_t kMapSig = 0x4000;

__host__ __device__ constexpr int16_t map_w(int N, int rr, int cc)
{
    return (rr >= 0 && rr < N && cc >= 0 && cc <= rr) ? (int16_t)(rr * (rr + 1) / 2 + cc)
                                                       : kMapZero;
}

// FP64 tile record: one entry per double (2 f64_rec_units(N) entries).
inline void cov_map_fp64(int N, int16_t *m)
{
    const int n = 2 * f64_rec_units(N), nt = f64_ntile(N), P = f64_pad(N), nbe = f64_nbe(N);
    const int nb = f64_nb(N), sig = f64_sig_double(N), lead = f64_lead_double(N);
    const int nl = f64_lead(N);
    for (int e = 0; e < n; ++e) {
        int16_t v = kMapZero;
        if (e < sig) {
            const int t = 2 * (e >> 5) + (e & 1), pos = (e >> 1) & 15;
            if (t < nt)
                v = map_w(N, 4 * f64_tile_r(N, t) + (pos & 3) - P,
                          4 * f64_tile_kb(N, t) + (pos >> 2) - P);
        } else if (e < lead) {
            const int g = (e - sig) / nbe, r = (e - sig) % nbe, k = 4 * r + g - P;
            if (k >= 0 && k < N) v = (int16_t)(kMapSig + k);
        } else if (e < lead + 4 * nbe * nl) {
            const int x = e - lead, c = x / (4 * nbe), g = (x / nbe) % 4, r = x % nbe;
            if (r < nb) v = map_w(N, 4 * r + g - P, c);
        }
        m[e] = v;
    }
}

// FP32 record, its W_q part: one entry per float (4 rec_w_units(ns) entries),
// A[v/4][lane][v%4] with lane 4 X + m holding pair t = 16 v + X.
inline void cov_map_fp32(int ns, int N, int16_t *m)
{
    const int P = fp32_pad(ns, N), np = fp32_npairs(ns);
    for (int v = 0; v < 4 * n_groups_from_ns(ns); ++v)
        for (int lane = 0; lane < 64; ++lane) {
            const int t = 16 * v + (lane >> 2), mm = lane & 3;
            int16_t x = kMapZero;
            if (t < np)
                x = map_w(N, 4 * fp32_pair_b(ns, t) + mm - P, fp32_pair_kp(ns, t) - P);
            m[((v >> 2) * 64 + lane) * 4 + (v & 3)] = x;
        }
}

// Split records, their fragments: eight entries per (fragment, lane), entry
// (f 64 + lane) 8 + e for element e of lane `lane`'s fragment f; kMapLo marks
// the low half of the split value (position 3 j + 2 of bin j).
constexpr int16_t kMapLo = 0x2000;
inline void cov_map_split(int N, int16_t *m)
{
    const int code = split_code(N);
    for (int g = 0; g < code_nb(code); ++g)
        for (int s = 0; s < code_steps(code, g); ++s) {
            const int f = code_frag(code, g, s);
            for (int lane = 0; lane < 64; ++lane) {
                const int row = split_row0(N, g) + (lane & 15);
                for (int e = 0; e < 8; ++e) {
                    const int p = 32 * s + 8 * (lane >> 4) + e, j = p / 3;
                    int16_t v = row < split_row0(N, g + 1) ? map_w(N, row, j) : kMapZero;
                    if (v != kMapZero && p % 3 == 2) v = (int16_t)(v | kMapLo);
                    m[(f * 64 + lane) * 8 + e] = v;
                }
            }
        }
}

// The maps of all three record forms, in the order FP64 | FP32 | split.
inline size_t cov_maps_size(int N, int ns)
{
    return (size_t)2 * f64_rec_units(N) + (size_t)4 * rec_w_units(ns) +
           (size_t)code_nfrag(split_code(N)) * 64 * 8;
}
inline void cov_maps_fill(int N, int ns, int16_t *m)
{
    cov_map_fp64(N, m);
    m += 2 * f64_rec_units(N);
    cov_map_fp32(ns, N, m);
    m += 4 * rec_w_units(ns);
    cov_map_split(N, m);
}

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
    double *S64 = nullptr;  // device [G][N]
    uint32_t forms = 0;
    double *W64 = nullptr;  // device [G][N(N+1)/2], packed lower W_q = L_q^{-1}
    uint4 *R32 = nullptr;   // device [G][rec_units(ns)] FP32-form records (see above)
    uint4 *RB16 = nullptr;  // device [G][split_rec_units] split-BF16 records
    uint4 *RH16 = nullptr;  // device [G][split_rec_units] split-FP16 records
    uint4 *R64 = nullptr;   // device [G][f64_rec_units] FP64 tile records (see above)
    double *off = nullptr;  // device [64] per-bin offset o (grid mean of S), zero past N
    double *dev = nullptr;  // device [64] per-bin max |S - o|
    int ed16 = 0;           // power-of-two scale of (d - o) in the split-FP16 form
    double *F64 = nullptr;  // device [N][N] fractional covariance of the last build
    double *LF64 = nullptr; // device [N][N] its Cholesky factor (universe generation)
    int lf_ok = 0;          // 1 if F is positive definite (LF64 valid)
    size_t bytes = 0;
    int ns = 0, ng = 0;     // FP32 fragment geometry
};

// ---- launchers (defined in the .hip files) ------------------------------
namespace fcx {

// Record a failure for fc_last_error on the calling thread; returns code.
int set_last_error(int code, const char *msg);

// Kernel timing (fc_profile_enable): while enabled, brackets the launches made
// in its scope by HIP events on the launch stream.
class ProfScope {
public:
    ProfScope(hipStream_t st, const char *name);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

private:
    hipStream_t st_;
    int slot_;
};

hipError_t launch_offset(const double *S64, int64_t G, int N, double *off, double *dev,
                         hipStream_t st);
// maps: a device copy of cov_maps_fill's table (cov_maps_size entries).
hipError_t launch_cov_build(const fc_grid *g, const double *F, const double *stat, int stat_mode,
                            uint32_t forms, const int16_t *maps, double *W64, uint4 *R64,
                            uint4 *R32, uint4 *RB16, uint4 *RH16, unsigned long long *bad_q,
                            hipStream_t st);
// The keyed scans cover the grid points [q0, q0 + nq) (nq = G: the whole grid)
// and merge into keys / chi2_p (see launch_init_keys).
hipError_t launch_scan_split(const fc_grid *g, bool fp16, int64_t K, const double *d,
                             const int64_t *p_idx, int64_t q0, int64_t nq,
                             unsigned long long *keys, double *chi2_p, hipStream_t st);
hipError_t launch_scan_fp32(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                            int64_t q0, int64_t nq, unsigned long long *keys, double *chi2_p,
                            hipStream_t st);
hipError_t launch_scan_fp32_points(const fc_grid *g, int64_t n_pts, const int64_t *p,
                                   const int64_t *seg_off, int64_t K, const double *d, int64_t q0,
                                   int64_t nq, const float *T, int64_t *tile_start,
                                   unsigned long long *keys, double *chi2_p, hipStream_t st);
// T [n_pts][nq][4 ns]: offset rows of the grid points [q0, q0 + nq).
hipError_t launch_offset_table(const fc_grid *g, int64_t n_pts, const int64_t *p, int64_t q0,
                               int64_t nq, float *T, hipStream_t st);
hipError_t launch_expand_segments(int64_t K, int64_t n_pts, const int64_t *seg_off,
                                  const int64_t *p, int64_t *p_idx, hipStream_t st);
// FP64 form; the chunk partials go to `scratch` (scratch_bytes, caller-owned)
// when it is given (fewer chunks if it is small), else to a stream-ordered
// allocation.
hipError_t launch_scan_fp64(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                            double *dchi2, double *chi2_min, int64_t *argmin, double *chi2_p,
                            hipStream_t st, Fp64Part *scratch = nullptr, size_t scratch_bytes = 0);
// keys = no value yet, chi2_p = chi2_p_fill (NaN for a one-call scan; 0 for
// the sliced-scan state, so that slices merge by summing chi2_p).
hipError_t launch_init_keys(int64_t K, unsigned long long *keys, double *chi2_p, hipStream_t st,
                            double chi2_p_fill = __builtin_nan(""));
// p_idx may be nullptr: then every universe's true point is p_uniform.
// chi2_min may alias keys (decoded in place); chi2_min and argmin may be
// nullptr (not written).  p_limit > 0: a true point
// outside [0, p_limit) gives dchi2 = NaN (its chi2_p was never written).
hipError_t launch_finalize(int64_t K, const int64_t *p_idx, const unsigned long long *keys,
                           double *chi2_min, int64_t *argmin, const double *chi2_p, double *dchi2,
                           hipStream_t st, int64_t p_uniform = -1, int64_t p_limit = 0);
hipError_t launch_inverse_cov(const fc_grid *g, int64_t q0, int64_t nq, double *out,
                              hipStream_t st);
hipError_t launch_crit(int64_t n_seg, const int64_t *seg_off, const double *x, int n_alpha,
                       const double *alpha, double *crit, int n_bins, double hist_hi,
                       int64_t *hist, hipStream_t st);

// One block's unit of scan work: a tile of universes of one request against
// a contiguous range of grid points of one grid.  fc_scan derives its items
// from the block index; the serving kernels read them from a table.
struct ScanItem {
    const uint4 *R;               // the grid's records (form layout)
    const double *d;              // universes [K][N] FP64
    const int64_t *p_idx;         // per-universe true points, or nullptr
    int64_t p;                    // the true point when p_idx is nullptr
    unsigned long long *keys;     // [K] packed (chi2 bits, q) minimum keys
    double *chi2_p;               // [K] chi2 at the true point
    const double *off;            // split forms: per-bin offset o
    int64_t K;                    // universes of the request
    int64_t u0;                   // first universe of the block's tile
    int64_t qb, qe;               // grid points [qb, qe)
    int32_t N;                    // bins
    int32_t ed;                   // split FP16: scale exponent of (d - o)
};

hipError_t launch_serve_fp32(int N, const ScanItem *items, int n_items, int *counter, int blocks,
                             hipStream_t st);
hipError_t launch_serve_split(int code, bool fp16, const ScanItem *items, int n_items,
                              int *counter, int blocks, hipStream_t st);
int serve_fp32_univ_per_item();
int serve_split_univ_per_item();
int serve_slots_fp32(int N);
int serve_slots_split(int code, bool fp16);

hipError_t launch_crit_gapped(int64_t n_seg, const int64_t *seg_lo, const int64_t *seg_hi,
                              const double *x, int n_alpha, const double *alpha, double *crit,
                              hipStream_t st);
hipError_t launch_select_ranks(int64_t n_seg, const int64_t *seg_lo, const int64_t *seg_hi,
                               const double *x, int n_q, const int64_t *ranks, double *out,
                               hipStream_t st);
int resident_slots(const void *kernel, int block_threads);
hipError_t fixed_run(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                     int max_iter, double *dchi2, double *chi2_min, int64_t *argmin,
                     double *chi2_p, int64_t *m_final, int32_t *iters, hipStream_t st);
int region_run(const fc_grid *g, int form, int64_t n_pts, const int64_t *pts_host, int64_t K0,
               int64_t K_max, double z, uint64_t seed, int n_alpha, const double *alpha,
               const double *dchi2_data, double *crit, uint8_t *accepted, int64_t *K_used,
               int32_t *n_rounds, double *n_evals, hipStream_t st, hipError_t *err);
hipError_t launch_chol_frac(const double *F, int N, double *LF, int *flag, hipStream_t st);
hipError_t launch_gen_universes(const fc_grid *g, int64_t n_pts, const int64_t *p,
                                const int64_t *seg_off, const int64_t *u_first, uint64_t seed,
                                int64_t K, double *d, int64_t *p_idx, int32_t *counts,
                                hipStream_t st);
hipError_t launch_data_scan(const fc_grid *g, const double *c, double *chi2,
                            unsigned long long *scratch, hipStream_t st);
hipError_t launch_accept(int64_t n_pts, const int64_t *p, const double *crit, int64_t stride,
                         const double *dchi2_data, int64_t G, uint8_t *accepted, hipStream_t st);

// Scan launch geometry chosen by the host: universe tiles x grid chunks.
struct ScanGeometry {
    int64_t n_utiles = 0;
    int64_t n_qchunks = 0;
    int64_t q_per_chunk = 0;
};
ScanGeometry scan_geometry(int64_t K, int64_t G, int slots, int univ_per_block);

}  // namespace fcx
