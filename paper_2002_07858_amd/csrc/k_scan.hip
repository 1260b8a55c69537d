// k_scan.hip -- the chi^2 grid scan (Eq. (1) inside Algorithm 1's loops).
//
// FP32 form (the hot kernel).  Eq. (1) is evaluated in factor form,
//     chi2(d, q) = ||W_q (d - S_q)||^2,   W_q = L_q^{-1} (lower triangular),
// which equals (d-S_q)^T Sigma_q^{-1} (d-S_q).  For a fixed q and a tile of
// universes this is a dense contraction Z = W_q R (R = bins x universes),
// done on the matrix cores with v_mfma_f32_4x4x1_16b_f32: one universe per
// lane, one bin per instruction, the 4-row slice of W_q broadcast to all 16
// lane blocks.  The 4-row granularity covers the lower triangle with little
// waste (N = 57: 1740 issued multiply-adds per evaluation for 1653 needed),
// and each lane ends with its own universe's rows, so chi2 is a lane-local
// sum of squares followed by a strict-"<" running minimum.  Vector
// instructions do not overlap the FP32 MFMAs on this chip, so the vector work
// around them (residuals, squares) is kept to few FP32 instructions.
//
// Work decomposition: a 256-thread block owns 256 universes (one per lane)
// and walks a contiguous range of grid points in list order.  Each lane
// keeps its universe's residual sources in registers; the block
// double-buffers one record per grid point in LDS (W_q slices, S_q and the
// correction C_q), bringing the next record in with direct global -> LDS
// loads while the waves contract the current one, with one barrier per grid
// point.  Ranges of the same universes are merged with a
// 64-bit atomicMin on keys (FP32 chi2 bits above q), which reproduces
// Algorithm 1's rule that the lowest q wins exact ties whatever the split.
#include "fc_internal.h"

#include <utility>

namespace fcx {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float pick(const float4 &v, int c)
{
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}

// Sixteen signal values, read through the scalar cache (uniform per wave).
struct Sig16 {
    float v[16];
};
typedef const __attribute__((address_space(4))) Sig16 *sig_ptr;
__device__ __forceinline__ Sig16 load_sig(sig_ptr p, int i)
{
    Sig16 r;
#pragma unroll
    for (int k = 0; k < 16; ++k) r.v[k] = p[i].v[k];
    return r;
}

// Per-universe state a lane carries through its range of grid points.  The
// universe is held as d = dh + dl: dh = float(d) and dl, the rest, as FP16
// scaled by a per-universe power of two 2^e (so that the largest |dl| 2^e
// lies in [2^14, 2^15)); dl 2^e keeps 11 bits, so d is carried to 35 bits,
// and the residual costs one subtraction and one mixed FP16/FP32 FMA.
template <int N>
struct Fp32Lane {
    float dh[N];
    uint32_t dl[(N + 1) / 2];  // dl 2^e as FP16, bins 2i (low half) and 2i+1 (high half)
    float dl_scale;            // 2^-e
    Sig16 s0;                  // the next grid point's first 16 signal values
    int64_t p_own;       // the universe's true point (-1: no universe)
    float best;          // running minimum and its grid point
    uint32_t qbest;
    float cp;            // chi2 at the true point, once seen
    bool have_cp;
};

// r = dl 2^-e + t with dl taken from one FP16 half of a packed register: the
// compiler folds the half selection and the conversion into one
// mixed-precision FMA (v_fma_mix_f32).
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
template <int HI>
__device__ __forceinline__ float fma_mix_dl(uint32_t dl2, float scale, float t)
{
    const half2_t h = __builtin_bit_cast(half2_t, dl2);
    return __builtin_fmaf((float)h[HI], scale, t);
}

// Per-grid-point operands: the A-register group being consumed and the next
// one (prefetched from LDS), the current and next 16 signal values (scalar
// registers) and the residual of the current bin.
constexpr int kResGroup = 8;  // residuals formed together (bins)

struct Fp32Ops {
    float4 a_cur, a_nxt;
    Sig16 s_cur, s_nxt;
    float r[kResGroup];  // residuals of the current group of bins
};

// Residual of real bin K into o.r[K % kResGroup], rotating the signal chunks
// when K starts a new one; with the last chunk in use, the next grid point's
// first chunk is fetched.
template <int N, int K>
__device__ __forceinline__ void fp32_residual(Fp32Ops &o, Fp32Lane<N> &L, sig_ptr sg,
                                              sig_ptr sg_next, bool more)
{
    constexpr int NCH = (N + 15) / 16;  // 16-value signal chunks
    if constexpr (K < N) {
        if constexpr (K % 16 == 0) {
            if constexpr (K > 0) o.s_cur = o.s_nxt;
            if constexpr (K / 16 + 1 < NCH) o.s_nxt = load_sig(sg, K / 16 + 1);
            if constexpr (K / 16 + 1 == NCH)
                if (more) L.s0 = load_sig(sg_next, 0);
        }
        const float t = L.dh[K] - o.s_cur.v[K % 16];
        o.r[K % kResGroup] = fma_mix_dl<K & 1>(L.dl[K / 2], L.dl_scale, t);
    }
}

// Pair T of the enumeration: rotate the A groups at a group boundary, form
// the residuals of a group of kResGroup bins at the first pair of the
// group's first bin, and issue one 4x4x1 MFMA whose A slice is broadcast
// from slot T % 16 of register T / 16.  Vector instructions do not overlap
// the FP32 MFMAs, and each switch from MFMAs to vector work costs about one
// MFMA's latency, so the residuals are formed in groups rather than one per
// bin.  Padded bins left of the shift (k' < P) are zero and generate no code.
template <int N, int T>
__device__ __forceinline__ void fp32_pair(v4f (&acc)[n_ksteps(N)], Fp32Ops &o, Fp32Lane<N> &L,
                                          const float4 *__restrict__ wl, sig_ptr sg,
                                          sig_ptr sg_next, bool more, int lane)
{
    constexpr int NS = n_ksteps(N), P = fp32_pad(NS, N);
    constexpr int KP = fp32_pair_kp(NS, T), B = fp32_pair_b(NS, T);
    constexpr int V = T / 16, NG = n_groups_from_ns(NS);
    if constexpr (T % 64 == 0 && T > 0) {
        o.a_cur = o.a_nxt;
        if constexpr (T / 64 + 1 < NG) o.a_nxt = wl[(T / 64 + 1) * 64 + lane];
    }
    if constexpr (KP >= P) {
        constexpr int K = KP - P;
        if constexpr (B == KP / 4 && K % kResGroup == 0) {
            static_assert(kResGroup == 8, "eight residuals per group");
            fp32_residual<N, K>(o, L, sg, sg_next, more);
            fp32_residual<N, K + 1>(o, L, sg, sg_next, more);
            fp32_residual<N, K + 2>(o, L, sg, sg_next, more);
            fp32_residual<N, K + 3>(o, L, sg, sg_next, more);
            fp32_residual<N, K + 4>(o, L, sg, sg_next, more);
            fp32_residual<N, K + 5>(o, L, sg, sg_next, more);
            fp32_residual<N, K + 6>(o, L, sg, sg_next, more);
            fp32_residual<N, K + 7>(o, L, sg, sg_next, more);
            // keep the group's vector work together, ahead of its MFMAs
            __builtin_amdgcn_sched_barrier(0);
        }
        acc[B] = __builtin_amdgcn_mfma_f32_4x4x1f32(pick(o.a_cur, V % 4), o.r[K % kResGroup],
                                                    acc[B], 4, T % 16, 0);
        // one group of bins at a time: keeps the scheduler from hoisting
        // operands of later bins (register pressure)
        if constexpr (B == NS - 1 && K % kResGroup == kResGroup - 1)
            __builtin_amdgcn_sched_barrier(0);
    }
}

template <int N, int... Ts>
__device__ __forceinline__ void fp32_pairs(v4f (&acc)[n_ksteps(N)], Fp32Ops &o, Fp32Lane<N> &L,
                                           const float4 *__restrict__ wl, sig_ptr sg,
                                           sig_ptr sg_next, bool more, int lane,
                                           std::integer_sequence<int, Ts...>)
{
    (fp32_pair<N, Ts>(acc, o, L, wl, sg, sg_next, more, lane), ...);
}

// chi2 = the lane's sum of squares (four FP32 chains over the row blocks; the
// P padding rows of block 0 are zero and skipped), folded into the running
// minimum with Algorithm 1's strict "<", and kept when q is the true point.
template <int NS, int P>
__device__ __forceinline__ void fp32_fold(const v4f (&acc)[NS], int64_t q, int64_t p_own,
                                          float &best, uint32_t &qbest, float &cp, bool &have_cp)
{
    float part[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        part[j] = (j >= P) ? acc[0][j] * acc[0][j] : 0.0f;
#pragma unroll
        for (int b = 1; b < NS; ++b) part[j] = fmaf(acc[b][j], acc[b][j], part[j]);
    }
    const float chi2 = (part[0] + part[1]) + (part[2] + part[3]);
    if (q == p_own) {
        cp = chi2;
        have_cp = true;
    }
    if (chi2 < best) {
        best = chi2;
        qbest = (uint32_t)q;
    }
}

// One grid point: contract the record in `cur`, fold chi2 into the running
// minimum, and (if more) bring the next record into `nxt`.  The two LDS
// buffers are separate objects so that the compiler can tell the copy into
// one from the reads of the other.  The signal values come from the record in
// global memory through scalar loads (read-only data, uniform addresses).
template <int N>
__device__ __forceinline__ void fp32_point(int64_t q, bool more, const uint4 *__restrict__ R32,
                                           const uint4 *cur, uint4 *nxt, Fp32Lane<N> &L)
{
    constexpr int NS = n_ksteps(N), P = fp32_pad(NS, N);
    constexpr int NWU = rec_w_units(NS);
    constexpr int REC = rec_units(NS);
    constexpr int THREADS = 64 * kWavesPerBlock;
    const int tid = threadIdx.x;
    const int lane = tid & 63;

    // signal values through the scalar cache (the first 16 were fetched during
    // the previous grid point); then the next record's copy, before the
    // contraction
    // the packed FP16 parts are re-presented to the compiler at every grid
    // point, so that their FP32 conversions stay inside the mixed FMAs
    // instead of being hoisted out of the grid loop into extra registers
#pragma unroll
    for (int i = 0; i < (N + 1) / 2; ++i) asm volatile("" : "+v"(L.dl[i]));
    Fp32Ops o;
    sig_ptr sg = (sig_ptr)(R32 + q * REC + NWU);  // Sh, real bins
    sig_ptr sg_next = (sig_ptr)(R32 + (q + 1) * REC + NWU);
    o.s_cur = L.s0;
    if (more) record_to_lds<REC, THREADS>(R32 + (q + 1) * REC, nxt, tid);
    __builtin_amdgcn_sched_barrier(0);

    const float4 *wl = reinterpret_cast<const float4 *>(cur);
    const float4 *cl = reinterpret_cast<const float4 *>(cur + NWU) + 16;  // C, 16 x float4
    // accumulators start at C_q (the same four rows in every lane)
    v4f acc[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) {
        const float4 cv = cl[b];
        acc[b] = v4f{cv.x, cv.y, cv.z, cv.w};
    }
    o.a_cur = wl[lane];
    if constexpr (n_groups_from_ns(NS) > 1) o.a_nxt = wl[64 + lane];
    fp32_pairs<N>(acc, o, L, wl, sg, sg_next, more, lane,
                  std::make_integer_sequence<int, fp32_npairs(NS)>{});

    fp32_fold<NS, P>(acc, q, L.p_own, L.best, L.qbest, L.cp, L.have_cp);

    if (more) wait_record_loads();
    __syncthreads();
}

// One work item (a tile of 256 universes x a range of grid points) in the
// residual form: d - S_q is formed per bin and grid point.
template <int N>
__device__ __forceinline__ void fp32_item(const ScanItem &it, uint4 *buf0, uint4 *buf1)
{
    constexpr int REC = rec_units(n_ksteps(N));  // A groups + 512 B of S and C
    constexpr int THREADS = 64 * kWavesPerBlock;
    static_assert(REC <= 3 * THREADS, "records of at most three 4 KB pieces");

    const uint4 *__restrict__ R32 = it.R;
    const double *__restrict__ d = it.d;
    const int64_t K = it.K;
    const int tid = threadIdx.x;
    const int64_t u = it.u0 + tid;  // this lane's universe
    const int64_t qb = it.qb, qe = it.qe;
    if (qb >= qe) return;  // uniform per block

    Fp32Lane<N> L;
    // residual sources d = dh + dl 2^-e (zero past K; lanes past K still take
    // part in the copies and barriers).  The rest d - dh is exact in FP64.
    float rest[N];
    float big = 0.0f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double v = (u < K) ? d[u * N + k] : 0.0;
        L.dh[k] = (float)v;
        rest[k] = (float)(v - (double)L.dh[k]);
        big = fmaxf(big, fabsf(rest[k]));
    }
    // largest |rest| 2^e in [2^14, 2^15); e clamped so that 2^-e stays a
    // normal FP32 number (rests that small are below FP16's reach and vanish)
    int e = (big > 0.0f) ? 14 - ilogbf(big) : 0;
    e = e < -100 ? -100 : (e > 100 ? 100 : e);
    L.dl_scale = ldexpf(1.0f, -e);
#pragma unroll
    for (int i = 0; i < (N + 1) / 2; ++i) {
        const _Float16 lo = (_Float16)ldexpf(rest[2 * i], e);
        const _Float16 hi = (2 * i + 1 < N) ? (_Float16)ldexpf(rest[2 * i + 1], e) : (_Float16)0.0f;
        L.dl[i] = (uint32_t)__builtin_bit_cast(uint16_t, lo) |
                  ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
    }
    L.p_own = (u < K) ? (it.p_idx ? it.p_idx[u] : it.p) : -1;
    L.best = __builtin_inff();
    L.qbest = 0xffffffffu;
    L.cp = 0.0f;
    L.have_cp = false;

    L.s0 = load_sig((sig_ptr)(R32 + qb * REC + rec_w_units(n_ksteps(N))), 0);
    record_to_lds<REC, THREADS>(R32 + qb * REC, buf0, tid);
    wait_record_loads();
    __syncthreads();
    // grid points in pairs so that each one's LDS buffer is fixed
    int64_t q = qb;
    for (; q + 1 < qe; q += 2) {
        fp32_point<N>(q, true, R32, buf0, buf1, L);
        fp32_point<N>(q + 1, q + 2 < qe, R32, buf1, buf0, L);
    }
    if (q < qe) fp32_point<N>(q, false, R32, buf0, buf1, L);

    if (u < K) {
        if (L.have_cp) it.chi2_p[u] = (double)L.cp;
        if (L.best < __builtin_inff()) {
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(L.best) << 32) | (unsigned long long)L.qbest;
            atomicMin(&it.keys[u], key);
        }
    }
}

// Offset form for a wave whose universes all belong to one true point p
// (Algorithm 1 runs per true point): with e = d - S_p rounded to FP32 once,
//     W_q (d - S_q) = W_q e + T_pq,    T_pq = W_q (S_p - S_q),
// and T_pq (FP64 arithmetic on the FP32 factor, rounded once) is the
// accumulators' start, read from a table built before the scan.  The MFMAs
// take e straight from registers, so the grid loop has no vector work besides
// the squares and the minimum.
template <int N>
struct Fp32Fast {
    float e[N];       // d - S_p
    int64_t p_own;    // -1: no universe
    float best;
    uint32_t qbest;
    float cp;
    bool have_cp;
};

// Copy one offset-table row (4 ns floats, 16-byte aligned) into the wave's
// LDS slot with direct global -> LDS loads, one 16-byte piece per lane.
template <int NS>
__device__ __forceinline__ void trow_to_lds(const float *__restrict__ row, float4 *dst_wave, int lane)
{
    if (lane < NS)
        __builtin_amdgcn_global_load_lds((const void *)(row + 4 * lane),
                                         (__attribute__((address_space(3))) void *)dst_wave, 16, 0,
                                         0);
}

template <int N, int T>
__device__ __forceinline__ void fp32_fast_pair(v4f (&acc)[n_ksteps(N)], float4 &a_cur, float4 &a_nxt,
                                               const Fp32Fast<N> &L, const float4 *__restrict__ wl,
                                               int lane)
{
    constexpr int NS = n_ksteps(N), P = fp32_pad(NS, N);
    constexpr int KP = fp32_pair_kp(NS, T), B = fp32_pair_b(NS, T);
    constexpr int V = T / 16, NG = n_groups_from_ns(NS);
    if constexpr (T % 64 == 0 && T > 0) {
        a_cur = a_nxt;
        if constexpr (T / 64 + 1 < NG) a_nxt = wl[(T / 64 + 1) * 64 + lane];
    }
    if constexpr (KP >= P) {
        acc[B] = __builtin_amdgcn_mfma_f32_4x4x1f32(pick(a_cur, V % 4), L.e[KP - P], acc[B], 4,
                                                    T % 16, 0);
        if constexpr (B == NS - 1 && (KP - P) % 8 == 7) __builtin_amdgcn_sched_barrier(0);
    }
}

template <int N, int... Ts>
__device__ __forceinline__ void fp32_fast_pairs(v4f (&acc)[n_ksteps(N)], float4 &a_cur,
                                                float4 &a_nxt, const Fp32Fast<N> &L,
                                                const float4 *__restrict__ wl, int lane,
                                                std::integer_sequence<int, Ts...>)
{
    (fp32_fast_pair<N, Ts>(acc, a_cur, a_nxt, L, wl, lane), ...);
}

template <int N>
__device__ __forceinline__ void fp32_fast_point(int64_t q, bool more, const uint4 *__restrict__ R32,
                                                const float *__restrict__ trow_q, const uint4 *cur,
                                                uint4 *nxt, const float4 *tcur, float4 *tnxt,
                                                Fp32Fast<N> &L)
{
    constexpr int NS = n_ksteps(N), P = fp32_pad(NS, N);
    constexpr int REC = rec_units(NS);
    constexpr int NR = 4 * NS;
    constexpr int THREADS = kPtsTile;
    const int tid = threadIdx.x;
    const int lane = tid & 63;

    if (more) {
        record_to_lds<REC, THREADS>(R32 + (q + 1) * REC, nxt, tid);
        if (tid < 64) trow_to_lds<NS>(trow_q + NR, tnxt, lane);
    }
    __builtin_amdgcn_sched_barrier(0);

    const float4 *wl = reinterpret_cast<const float4 *>(cur);
    v4f acc[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) {
        const float4 tv = tcur[b];
        acc[b] = v4f{tv.x, tv.y, tv.z, tv.w};
    }
    float4 a_cur = wl[lane], a_nxt = a_cur;
    if constexpr (n_groups_from_ns(NS) > 1) a_nxt = wl[64 + lane];
    fp32_fast_pairs<N>(acc, a_cur, a_nxt, L, wl, lane,
                       std::make_integer_sequence<int, fp32_npairs(NS)>{});
    fp32_fold<NS, P>(acc, q, L.p_own, L.best, L.qbest, L.cp, L.have_cp);

    if (more) wait_record_loads();
    __syncthreads();
}

template <int N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_scan_fp32(
    const uint4 *__restrict__ R32, const double *__restrict__ d,
    const int64_t *__restrict__ p_idx, int64_t K, int64_t q_lo, int64_t q_hi, int64_t n_utiles,
    int64_t q_per_chunk, unsigned long long *__restrict__ keys, double *__restrict__ chi2_p)
{
    __shared__ uint4 buf0[rec_units(n_ksteps(N))], buf1[rec_units(n_ksteps(N))];
    ScanItem it;
    it.R = R32;
    it.d = d;
    it.p_idx = p_idx;
    it.p = -1;
    it.keys = keys;
    it.chi2_p = chi2_p;
    it.off = nullptr;
    it.K = K;
    it.N = N;
    it.ed = 0;
    const int64_t utile = blockIdx.x % n_utiles;
    const int64_t qchunk = blockIdx.x / n_utiles;
    it.u0 = utile * (int64_t)kFp32UnivPerBlock;
    it.qb = q_lo + qchunk * q_per_chunk;
    it.qe = (it.qb + q_per_chunk < q_hi) ? it.qb + q_per_chunk : q_hi;
    fp32_item<N>(it, buf0, buf1);
}

// Serving: a persistent-style launch over a table of items (any mix of
// requests and grids with this bin count).  Resident blocks take items in
// turn from an atomic counter until the table is exhausted; the table is
// finite and fixed at launch, so every block reaches the exit.
template <int N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_serve_fp32(
    const ScanItem *__restrict__ items, int n_items, int *__restrict__ counter)
{
    __shared__ uint4 buf0[rec_units(n_ksteps(N))], buf1[rec_units(n_ksteps(N))];
    __shared__ int cur;
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
        __syncthreads();
        const int i = cur;
        __syncthreads();
        if (i >= n_items) break;
        fp32_item<N>(items[i], buf0, buf1);
        __syncthreads();
    }
}

// Scan of universes grouped by true point, offset form throughout.  Tiles of
// B = kPtsTile universes never straddle segments: segment s owns the dense
// tile ids [tile_start[s], tile_start[s+1]), tile_start[s+1] - tile_start[s] =
// ceil(len_s / B) (a prefix sum built before the launch), all below
// floor(K / B) + n_pts.  Each block scans one tile (its waves share the true
// point, so one offset-table row per grid point serves them all) over a range
// of grid points.  Blocks are dispatched round-robin over the 8 XCDs (block b
// runs on XCD b mod 8), so block b = xcd + 8 (m + 8 (j + J c)) is given tile
// 8 (xcd + 8 j) + m of grid chunk c: eight consecutive tiles (a segment's,
// mostly) run on one XCD at the same time and share its L2 for the offset
// rows and the records, and the XCDs get equal shares of the tiles.
// The grid points scanned are [q_lo, q_hi): the whole grid, or one slice of it
// when the grid is split over several launches or devices.  Segments whose
// true point is outside the grid do nothing.
template <int N>
__global__ __launch_bounds__(kPtsTile) __attribute__((amdgpu_waves_per_eu(2))) void k_scan_fp32_pts(
    const uint4 *__restrict__ R32, const double *__restrict__ S64, const double *__restrict__ d,
    int64_t G, int64_t n_pts, const int64_t *__restrict__ p, const int64_t *__restrict__ seg_off,
    const int64_t *__restrict__ tile_start, const float *__restrict__ T, int64_t groups_per_xcd,
    int64_t q_lo, int64_t q_hi, int64_t q_per_chunk, int64_t K,
    unsigned long long *__restrict__ keys, double *__restrict__ chi2_p)
{
    constexpr int NS = n_ksteps(N);
    constexpr int REC = rec_units(NS);
    constexpr int NR = 4 * NS;
    constexpr int THREADS = kPtsTile;
    __shared__ uint4 buf0[REC], buf1[REC];
    __shared__ float4 tb0[16], tb1[16];
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % 8, k = b / 8;
    const int64_t member = k % 8, rest = k / 8;
    const int64_t group = xcd + 8 * (rest % groups_per_xcd);
    const int64_t tile = 8 * group + member;
    const int64_t qb = q_lo + (rest / groups_per_xcd) * q_per_chunk;
    const int64_t qe = (qb + q_per_chunk < q_hi) ? qb + q_per_chunk : q_hi;
    if (tile >= tile_start[n_pts]) return;  // uniform per block
    // the tile's segment: the largest s with tile_start[s] <= tile (uniform)
    int64_t lo = 0, hi = n_pts - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int64_t seg = lo;
    const int64_t i = tile - tile_start[seg];
    const int64_t s0 = seg_off[seg], s1 = seg_off[seg + 1];
    const int64_t pp = p[seg];
    if (qb >= qe || pp < 0 || pp >= G) return;  // uniform per block
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int64_t u = s0 + kPtsTile * i + tid;
    // (the row must also lie in [0, K): offsets that break their contract
    // read and write nothing outside the arrays)
    const bool act = u < s1 && u >= 0 && u < K;

    Fp32Fast<N> L;
    const double *__restrict__ sp = S64 + pp * N;  // uniform: scalar loads
#pragma unroll
    for (int k = 0; k < N; ++k) L.e[k] = act ? (float)(d[u * N + k] - sp[k]) : 0.0f;
    L.p_own = act ? pp : -1;
    L.best = __builtin_inff();
    L.qbest = 0xffffffffu;
    L.cp = 0.0f;
    L.have_cp = false;
    // offset rows of this segment: one per grid point of [q_lo, q_hi)
    const float *__restrict__ trow = T + (seg * (q_hi - q_lo) + (qb - q_lo)) * NR;

    record_to_lds<REC, THREADS>(R32 + qb * REC, buf0, tid);
    if (tid < 64) trow_to_lds<NS>(trow, tb0, lane);
    wait_record_loads();
    __syncthreads();
    int64_t q = qb;
    for (; q + 1 < qe; q += 2, trow += 2 * NR) {
        fp32_fast_point<N>(q, true, R32, trow, buf0, buf1, tb0, tb1, L);
        fp32_fast_point<N>(q + 1, q + 2 < qe, R32, trow + NR, buf1, buf0, tb1, tb0, L);
    }
    if (q < qe) fp32_fast_point<N>(q, false, R32, trow, buf0, buf1, tb0, tb1, L);

    if (act) {
        if (L.have_cp) chi2_p[u] = (double)L.cp;
        if (L.best < __builtin_inff()) {
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(L.best) << 32) | (unsigned long long)L.qbest;
            atomicMin(&keys[u], key);
        }
    }
}

__global__ __launch_bounds__(256) void k_init_keys(int64_t K, unsigned long long *__restrict__ keys,
                                                  double *__restrict__ chi2_p, double chi2_p_fill)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= K) return;
    keys[u] = kKeyNone;
    chi2_p[u] = chi2_p_fill;
}

// Decode the keys.  chi2_min may be the key buffer itself (decoded in place:
// each thread reads its key before it writes the same element); chi2_min and
// argmin may be nullptr.  A universe
// with no finite chi2 keeps Algorithm 1's initial state and gets a NaN dchi2,
// and so does one whose true point is outside [0, p_limit) when p_limit > 0.
__global__ __launch_bounds__(256) void k_finalize(int64_t K, const int64_t *__restrict__ p_idx,
                                                 int64_t p_uniform, int64_t p_limit,
                                                 const unsigned long long *keys, double *chi2_min,
                                                 int64_t *__restrict__ argmin,
                                                 const double *__restrict__ chi2_p,
                                                 double *__restrict__ dchi2)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= K) return;
    const unsigned long long key = keys[u];
    const uint32_t hi = (uint32_t)(key >> 32);
    double cmin, dc;
    int64_t am;
    if (hi >= 0x7f800000u) {  // no chi2 < +inf was seen: Algorithm 1's initial state
        cmin = __builtin_inf();
        am = p_idx ? p_idx[u] : p_uniform;
        dc = __builtin_nan("");
    } else {
        cmin = (double)__uint_as_float(hi);
        am = (int64_t)(uint32_t)(key & 0xffffffffu);
        dc = chi2_p[u] - cmin;
        if (p_limit > 0) {
            const int64_t pu = p_idx ? p_idx[u] : p_uniform;
            if (pu < 0 || pu >= p_limit) dc = __builtin_nan("");
        }
    }
    if (chi2_min) chi2_min[u] = cmin;
    if (argmin) argmin[u] = am;
    dchi2[u] = dc;
}

// ---------------------------------------------------------------------------
// Resident block slots of a kernel on the current device: CUs x blocks per CU
// from the occupancy calculator.
int resident_slots(const void *kernel, int block_threads)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 512;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block_threads, 0) !=
            hipSuccess ||
        per_cu <= 0)
        per_cu = 2;
    return cus * per_cu;
}

// Pick the number of grid chunks so that tiles x chunks fills the resident
// block slots with the smallest tail: minimise ceil(tiles*c/slots)/c, with a
// small charge per chunk.  With few tiles (a small K) every chunk count up to
// G / min_chunk fits in one round and the most chunks win, so min_chunk sets
// how far a small scan spreads over the CUs; at large K the tail term decides.
ScanGeometry scan_geometry(int64_t K, int64_t G, int slots, int univ_per_block)
{
    ScanGeometry sg;
    sg.n_utiles = (K + univ_per_block - 1) / univ_per_block;
    const int64_t min_chunk = 8;
    int64_t cmax = G / min_chunk;
    if (cmax < 1) cmax = 1;
    if (cmax > 256) cmax = 256;
    // keep blocks * 256 work-items well inside the 32-bit dispatch size
    const int64_t max_blocks = int64_t(1) << 23;
    const int64_t cfit = max_blocks / (sg.n_utiles > 0 ? sg.n_utiles : 1);
    if (cmax > cfit) cmax = cfit > 0 ? cfit : 1;
    double best = 1e300;
    int64_t bestc = 1;
    for (int64_t c = 1; c <= cmax; ++c) {
        const int64_t units = sg.n_utiles * c;
        const double rounds = (double)((units + slots - 1) / slots);
        const double cost = rounds / (double)c * (1.0 + 0.002 * (double)c);  // chunk overhead
        if (cost < best * (1.0 - 1e-9)) {
            best = cost;
            bestc = c;
        }
    }
    sg.q_per_chunk = (G + bestc - 1) / bestc;
    sg.n_qchunks = (G + sg.q_per_chunk - 1) / sg.q_per_chunk;
    return sg;
}

template <int N>
static hipError_t launch_fp32_n(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                                int64_t q0, int64_t nq, unsigned long long *keys, double *chi2_p,
                                hipStream_t st)
{
    // resident block slots: queried once per instantiation (thread-safe)
    static const int slots =
        resident_slots(reinterpret_cast<const void *>(&k_scan_fp32<N>), 64 * kWavesPerBlock);
    ScanGeometry sg = scan_geometry(K, nq, slots, kFp32UnivPerBlock);
    // then chunks of at most kFp32ChunkMax points, as far as the dispatch size
    // allows, as in the points form (c3: 1.59 s against 1.68 s, c5 0.5 %
    // faster; the same results bit for bit)
    constexpr int64_t kFp32ChunkMax = 2048;
    if (sg.q_per_chunk > kFp32ChunkMax) {
        const int64_t cap = (int64_t(1) << 23) / (sg.n_utiles > 0 ? sg.n_utiles : 1);
        int64_t nc = (nq + kFp32ChunkMax - 1) / kFp32ChunkMax;
        if (nc > cap) nc = cap;
        if (nc > sg.n_qchunks) {
            sg.q_per_chunk = (nq + nc - 1) / nc;
            sg.n_qchunks = (nq + sg.q_per_chunk - 1) / sg.q_per_chunk;
        }
    }
    const int64_t blocks = sg.n_utiles * sg.n_qchunks;
    ProfScope prof(st, "k_scan_fp32");
    hipLaunchKernelGGL((k_scan_fp32<N>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, st,
                       g->R32, d, p_idx, K, q0, q0 + nq, sg.n_utiles, sg.q_per_chunk, keys, chi2_p);
    return hipGetLastError();
}

// Dense tile ids of the points scan: tile_start[0] = 0, tile_start[s+1] =
// tile_start[s] + ceil((seg_off[s+1] - seg_off[s]) / kPtsTile).  One block;
// segments in chunks of 1024 with a running carry.
__global__ __launch_bounds__(1024) void k_tile_prefix(int64_t n_pts,
                                                      const int64_t *__restrict__ seg_off,
                                                      int64_t *__restrict__ tile_start)
{
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    int64_t carry = 0;
    if (tid == 0) tile_start[0] = 0;
    for (int64_t base = 0; base < n_pts; base += 1024) {
        const int64_t s = base + tid;
        int64_t v = 0;
        if (s < n_pts) {
            const int64_t len = seg_off[s + 1] - seg_off[s];
            v = len > 0 ? (len + kPtsTile - 1) / kPtsTile : 0;
        }
        part[tid] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan (Hillis-Steele)
            const int64_t add = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += add;
            __syncthreads();
        }
        if (s < n_pts) tile_start[s + 1] = carry + part[tid];
        carry += part[1023];
        __syncthreads();
    }
}

template <int N>
static hipError_t launch_fp32_pts_n(const fc_grid *g, int64_t n_pts, const int64_t *p,
                                    const int64_t *seg_off, int64_t K, const double *d, int64_t q0,
                                    int64_t nq, const float *T, int64_t *tile_start,
                                    unsigned long long *keys, double *chi2_p, hipStream_t st)
{
    // resident block slots: queried once per instantiation (thread-safe)
    static const int slots =
        resident_slots(reinterpret_cast<const void *>(&k_scan_fp32_pts<N>), kPtsTile);
    const int64_t max_tiles = K / kPtsTile + n_pts;  // bound on the dense tile count
    const int64_t groups_per_xcd = (max_tiles + 63) / 64;
    const int64_t n_tiles = 64 * groups_per_xcd;    // blocks per grid chunk
    ScanGeometry sg = scan_geometry(max_tiles * kPtsTile, nq, slots, kPtsTile);
    // then shorter chunks, of at most kPtsChunkMax points, as far as the
    // dispatch size allows: the tiles that share a chunk start together and
    // stay close, so the L2 serves the later readers of each record (c5:
    // 4.65 s against 4.81 s for the whole call, the same results bit for bit)
    constexpr int64_t kPtsChunkMax = 2048;
    if (sg.q_per_chunk > kPtsChunkMax) {
        const int64_t cap = (int64_t(1) << 23) / n_tiles;
        int64_t nc = (nq + kPtsChunkMax - 1) / kPtsChunkMax;
        if (nc > cap) nc = cap;
        if (nc > sg.n_qchunks) {
            sg.q_per_chunk = (nq + nc - 1) / nc;
            sg.n_qchunks = (nq + sg.q_per_chunk - 1) / sg.q_per_chunk;
        }
    }
    const int64_t blocks = n_tiles * sg.n_qchunks;
    hipLaunchKernelGGL(k_tile_prefix, dim3(1), dim3(1024), 0, st, n_pts, seg_off, tile_start);
    ProfScope prof(st, "k_scan_fp32_pts");
    hipLaunchKernelGGL((k_scan_fp32_pts<N>), dim3((unsigned)blocks), dim3(kPtsTile), 0,
                       st, g->R32, g->S64, d, g->G, n_pts, p, seg_off, tile_start, T, groups_per_xcd,
                       q0, q0 + nq, sg.q_per_chunk, K, keys, chi2_p);
    return hipGetLastError();
}

// Offset table of the FP32 offset form: T[pt][q - q_lo][r'] = sum_k' W'_q[r'][k']
// (S_p - S_q)[k' - P] for the true point p = p[pt] of every segment and every
// grid point q of [q_lo, q_lo + nq), in FP64
// arithmetic on the FP32 factor as the scan uses it (padded rows r' < 4 ns),
// rounded once to FP32; rows of an out-of-range p are zero (such segments take
// the residual form).  One block per grid point (grid-stride): the record's A
// slices are expanded into the transposed dense factor W'^T in LDS (zero above
// the diagonal), and each thread accumulates one 4-row block of one segment,
// bin by bin, from float4 columns of W'^T.
template <int N>
__global__ __launch_bounds__(256) void k_offset_table(const uint4 *__restrict__ R32,
                                                      const double *__restrict__ S64, int64_t G,
                                                      int64_t q_lo, int64_t nq, int64_t n_pts,
                                                      const int64_t *__restrict__ p,
                                                      float *__restrict__ T)
{
    constexpr int NS = n_ksteps(N), P = fp32_pad(NS, N), NR = 4 * NS;
    constexpr int REC = rec_units(NS), NP = fp32_npairs(NS), NG = n_groups_from_ns(NS);
    __shared__ float4 Wt[NR * NS];  // Wt[k'][b] = W'[4b .. 4b+3][k']
    __shared__ double Sq[NR];
    __shared__ unsigned char pk[NP], pb[NP];
    const int tid = threadIdx.x;
    if (tid == 0) {
        int t = 0;
        for (int kp = 0; kp < NR; ++kp)
            for (int b = kp / 4; b < NS; ++b, ++t) {
                pk[t] = (unsigned char)kp;
                pb[t] = (unsigned char)b;
            }
    }
    __syncthreads();
    float *wt = reinterpret_cast<float *>(Wt);
    for (int64_t j = blockIdx.x; j < nq; j += gridDim.x) {
        const int64_t q = q_lo + j;
        for (int i = tid; i < NR * NR; i += blockDim.x) wt[i] = 0.0f;
        for (int i = tid; i < NR; i += blockDim.x) Sq[i] = (i >= P) ? S64[q * N + (i - P)] : 0.0;
        __syncthreads();
        const float *rec = reinterpret_cast<const float *>(R32 + q * REC);
        // float f of the A part: register v = 4 (f / 256) + f % 4, lane (f / 4) % 64
        for (int f = tid; f < NG * 256; f += blockDim.x) {
            const int v = 4 * (f / 256) + (f & 3), ln = (f >> 2) & 63;
            const int t = 16 * v + (ln >> 2);
            if (t < NP) wt[pk[t] * NR + 4 * pb[t] + (ln & 3)] = rec[f];
        }
        __syncthreads();
        // one thread per (segment, 4-row block): few segments still use the
        // whole block, and a row's sum runs over k' in ascending order
        for (int64_t w = tid; w < n_pts * NS; w += blockDim.x) {
            const int64_t pt = w / NS;
            const int b = (int)(w - pt * NS);
            const int64_t pp = p[pt];
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            if (pp >= 0 && pp < G) {
                const double *sp = S64 + pp * N - P;
                for (int kp = P; kp < NR; ++kp) {
                    const double dk = sp[kp] - Sq[kp];
                    const float4 wv = Wt[kp * NS + b];
                    a0 = fma((double)wv.x, dk, a0);
                    a1 = fma((double)wv.y, dk, a1);
                    a2 = fma((double)wv.z, dk, a2);
                    a3 = fma((double)wv.w, dk, a3);
                }
            }
            reinterpret_cast<float4 *>(T + (pt * nq + j) * NR)[b] =
                make_float4((float)a0, (float)a1, (float)a2, (float)a3);
        }
        __syncthreads();
    }
}

// Segment expansion: universe u of segment s = max{k : seg_off[k] <= u} gets
// p_idx[u] = p[s].
__global__ __launch_bounds__(256) void k_expand_segments(int64_t K, int64_t n_pts,
                                                         const int64_t *__restrict__ seg_off,
                                                         const int64_t *__restrict__ p,
                                                         int64_t *__restrict__ p_idx)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < K;
         u += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n_pts - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (seg_off[mid] <= u)
                lo = mid;
            else
                hi = mid - 1;
        }
        p_idx[u] = p[lo];
    }
}

template <int N>
static hipError_t launch_offset_table_n(const fc_grid *g, int64_t n_pts, const int64_t *p,
                                        int64_t q0, int64_t nq, float *T, hipStream_t st)
{
    const int64_t blocks = nq < 65536 ? nq : 65536;
    ProfScope prof(st, "k_offset_table");
    hipLaunchKernelGGL((k_offset_table<N>), dim3((unsigned)blocks), dim3(256), 0, st, g->R32, g->S64,
                       g->G, q0, nq, n_pts, p, T);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_serve_fp32_n(const ScanItem *items, int n_items, int *counter, int blocks,
                                      hipStream_t st)
{
    hipLaunchKernelGGL((k_serve_fp32<N>), dim3((unsigned)blocks), dim3(256), 0, st, items, n_items,
                       counter);
    return hipGetLastError();
}

template <int N>
static int serve_slots_fp32_n()
{
    // resident block slots: queried once per instantiation (thread-safe)
    static const int slots =
        resident_slots(reinterpret_cast<const void *>(&k_serve_fp32<N>), 256);
    return slots;
}

int serve_fp32_univ_per_item() { return kFp32UnivPerBlock; }

// One instantiation per bin count: the padding shift and the skipped pairs
// are compile-time constants of the kernel.
#define FC_EACH_N(X)                                                                            \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)       \
    X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) \
    X(32) X(33) X(34) X(35) X(36) X(37) X(38) X(39) X(40) X(41) X(42) X(43) X(44) X(45) X(46) \
    X(47) X(48) X(49) X(50) X(51) X(52) X(53) X(54) X(55) X(56) X(57) X(58) X(59) X(60) X(61) \
    X(62) X(63) X(64)

hipError_t launch_serve_fp32(int N, const ScanItem *items, int n_items, int *counter, int blocks,
                             hipStream_t st)
{
    switch (N) {
#define FC_CASE(n) \
    case n: return launch_serve_fp32_n<n>(items, n_items, counter, blocks, st);
        FC_EACH_N(FC_CASE)
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

int serve_slots_fp32(int N)
{
    switch (N) {
#define FC_CASE(n) \
    case n: return serve_slots_fp32_n<n>();
        FC_EACH_N(FC_CASE)
#undef FC_CASE
    default: return 512;
    }
}

hipError_t launch_scan_fp32(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                            int64_t q0, int64_t nq, unsigned long long *keys, double *chi2_p,
                            hipStream_t st)
{
    switch (g->N) {
#define FC_CASE(n) \
    case n: return launch_fp32_n<n>(g, K, d, p_idx, q0, nq, keys, chi2_p, st);
        FC_EACH_N(FC_CASE)
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_scan_fp32_points(const fc_grid *g, int64_t n_pts, const int64_t *p,
                                   const int64_t *seg_off, int64_t K, const double *d, int64_t q0,
                                   int64_t nq, const float *T, int64_t *tile_start,
                                   unsigned long long *keys, double *chi2_p, hipStream_t st)
{
    switch (g->N) {
#define FC_CASE(n)                                                                             \
    case n:                                                                                    \
        return launch_fp32_pts_n<n>(g, n_pts, p, seg_off, K, d, q0, nq, T, tile_start, keys, \
                                    chi2_p, st);
        FC_EACH_N(FC_CASE)
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_offset_table(const fc_grid *g, int64_t n_pts, const int64_t *p, int64_t q0,
                               int64_t nq, float *T, hipStream_t st)
{
    switch (g->N) {
#define FC_CASE(n) \
    case n: return launch_offset_table_n<n>(g, n_pts, p, q0, nq, T, st);
        FC_EACH_N(FC_CASE)
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_expand_segments(int64_t K, int64_t n_pts, const int64_t *seg_off,
                                  const int64_t *p, int64_t *p_idx, hipStream_t st)
{
    int64_t blocks = (K + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_expand_segments, dim3((unsigned)blocks), dim3(256), 0, st, K, n_pts, seg_off,
                       p, p_idx);
    return hipGetLastError();
}
#undef FC_EACH_N

hipError_t launch_init_keys(int64_t K, unsigned long long *keys, double *chi2_p, hipStream_t st,
                            double chi2_p_fill)
{
    const int64_t blocks = (K + 255) / 256;
    hipLaunchKernelGGL(k_init_keys, dim3((unsigned)blocks), dim3(256), 0, st, K, keys, chi2_p,
                       chi2_p_fill);
    return hipGetLastError();
}

hipError_t launch_finalize(int64_t K, const int64_t *p_idx, const unsigned long long *keys,
                           double *chi2_min, int64_t *argmin, const double *chi2_p, double *dchi2,
                           hipStream_t st, int64_t p_uniform, int64_t p_limit)
{
    const int64_t blocks = (K + 255) / 256;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)blocks), dim3(256), 0, st, K, p_idx, p_uniform,
                       p_limit, keys, chi2_min, argmin, chi2_p, dchi2);
    return hipGetLastError();
}

}  // namespace fcx
