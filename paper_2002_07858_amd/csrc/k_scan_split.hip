// k_scan_split.hip -- the chi^2 scan in the split-precision forms.
//
// Same statistic as the FP32 form (Eq. (1) in factor form inside Algorithm
// 1's loops), evaluated on the 16-bit matrix cores: every FP32 operand is
// written as hi + lo (BF16 or FP16) and a product as hi*hi + hi*lo + lo*hi,
// accumulated in FP32 by v_mfma_f32_16x16x32_{bf16,f16}.  By linearity
//     2^(eq+ed) z = [2^eq W_q] [2^ed (d - o)] - 2^(eq+ed) W_q (S_q - o),
// the universes 2^ed (d - o) are split once into registers and the per-point
// vector -2^(eq+ed) u_q, u_q = W_q (S_q - o), comes precomputed (FP64) with
// the record as the accumulators' initial value, so the loop over grid points
// does no per-universe residual work: MFMAs, then one square per z value and
// one power-of-two rescale per universe.  The three products of a bin are
// adjacent positions of one k sequence (layout in fc_internal.h), so the B
// fragments hold d_hi, d_lo, d_hi, d_hi, d_lo, ... and each row group issues
// ceil(3 (last row + 1) / 32) MFMAs per column block.
//
// Work decomposition as in the FP32 form: a 256-thread block owns 4 waves x
// 16*NC universes and walks a chunk of grid points, double-buffering one
// record per point in LDS; chunks merge through the packed-key atomicMin.
#include "fc_internal.h"

namespace fcx {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <bool FP16>
__device__ __forceinline__ v4f mfma16x16x32(const uint4 &a, const uint4 &b, const v4f &c)
{
    if constexpr (FP16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

template <bool FP16>
__device__ __forceinline__ void split8(const float (&x)[8], uint4 &hi, uint4 &lo)
{
    if constexpr (FP16) {
        f16x8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            h[e] = (_Float16)x[e];
            l[e] = (_Float16)(x[e] - (float)h[e]);
        }
        hi = __builtin_bit_cast(uint4, h);
        lo = __builtin_bit_cast(uint4, l);
    } else {
        bf16x8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            h[e] = (__bf16)x[e];
            l[e] = (__bf16)(x[e] - (float)h[e]);
        }
        hi = __builtin_bit_cast(uint4, h);
        lo = __builtin_bit_cast(uint4, l);
    }
}

// The k-sequence entry of position p = 3 j + t: the low half of bin j's split
// for t = 1, the high half otherwise; each 16-bit half of a 32-bit word picked
// by its own flag.
__device__ __forceinline__ uint4 pick_lo(const uint4 &hi, const uint4 &lo, uint32_t lomask)
{
    uint32_t w[4];
    const uint32_t *ph = reinterpret_cast<const uint32_t *>(&hi);
    const uint32_t *pl = reinterpret_cast<const uint32_t *>(&lo);
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const uint32_t m = ((lomask >> (2 * h)) & 1u ? 0x0000ffffu : 0u) |
                           ((lomask >> (2 * h + 1)) & 1u ? 0xffff0000u : 0u);
        w[h] = (ph[h] & ~m) | (pl[h] & m);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// LDS fragment reads kept in flight ahead of the MFMAs that use them (c5:
// FP16 1.59 s with one against 1.63 s with two, BF16 1.53 s either way
// within 0.4 %; three is slower for both).
template <bool FP16>
constexpr int kFragAhead = FP16 ? 1 : 2;

// Per-universe state a wave carries through its range of grid points.
template <int SM, int NC>
struct SplitLane {
    uint4 dx[NC][SM];   // B operands: the k sequence of 2^(ed - eu) (d - o), split
    uint32_t eu_pk;     // per-universe exponents eu (FP16 range), 8 bits per
                        // column block; 0 unless far outside the grid's range
    int e_own;          // eu of the universe this lane owns after the reduction
    bool scaled;        // some universe of the wave has eu != 0 (wave-uniform)
    int64_t p_own;
    float best;
    uint32_t qbest;
    float cp;
    bool have_cp;
};

// One grid point: contract the record in `cur`, fold chi2 into the running
// minimum, and (if more) bring the next record into `nxt` (separate LDS
// objects, see the FP32 form).
template <int CODE, int NC, bool FP16, bool SCALED>
__device__ __forceinline__ void split_point(int64_t q, bool more, const uint4 *__restrict__ R16,
                                            const uint4 *cur, uint4 *nxt,
                                            SplitLane<code_smax(CODE), NC> &L)
{
    constexpr int NB = code_nb(CODE);
    constexpr int REC = code_rec_units(CODE);
    constexpr int UU = code_u_unit(CODE);
    constexpr int SU = code_scale_unit(CODE);
    constexpr int THREADS = 64 * kWavesPerBlock;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int grp = lane >> 4;

    if (more) record_to_lds<REC, THREADS>(R16 + (q + 1) * REC, nxt, tid);
    __builtin_amdgcn_sched_barrier(0);  // issue the copy before the contraction

    // every accumulator starts at -2^(eq+ed-eu) u_q for its rows (the record
    // holds -2^(eq+ed) u_q; eu = 0 unless the wave holds a universe far outside
    // the grid's range, which only then costs the rescale)
    const float4 *ul = reinterpret_cast<const float4 *>(cur + UU) + grp * 4;
    v4f acc[NC][NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const float4 c0 = ul[b];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c][b] = v4f{c0.x, c0.y, c0.z, c0.w};
    }
    if constexpr (SCALED) {
        {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int e = (int)((L.eu_pk >> (8 * c)) & 255u);
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[c][b][j] = ldexpf(acc[c][b][j], -e);
            }
        }
    }
    // fragments in issue order, each read kFragAhead<FP16> fragments before its
    // MFMAs (a fence per fragment keeps the reads from all being hoisted, which
    // would hold every fragment of the record in registers at once)
    constexpr int NF = code_nfrag(CODE);
    uint4 w[NF];
#pragma unroll
    for (int i = 0; i < kFragAhead<FP16> && i < NF; ++i)
        w[i] = cur[code_frag(CODE, code_issue_g(CODE, i), code_issue_s(CODE, i)) * 64 + lane];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        if (i + kFragAhead<FP16> < NF) {
            const int ia = i + kFragAhead<FP16>;
            w[ia] = cur[code_frag(CODE, code_issue_g(CODE, ia), code_issue_s(CODE, ia)) * 64 + lane];
        }
        const int s = code_issue_s(CODE, i), b = code_issue_g(CODE, i);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c][b] = mfma16x16x32<FP16>(w[i], L.dx[c][s], acc[c][b]);
        __builtin_amdgcn_sched_barrier(0);
    }

    // acc = 2^(eq+ed) z: squared and summed per universe column
    const float unscale = __uint_as_float(cur[SU].x);
    float part[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        float blk[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            float a = acc[c][b][0] * acc[c][b][0];
#pragma unroll
            for (int j = 1; j < 4; ++j) a = fmaf(acc[c][b][j], acc[c][b][j], a);
            blk[b] = a;
        }
        if constexpr (NB == 4)
            part[c] = (blk[0] + blk[1]) + (blk[2] + blk[3]);
        else if constexpr (NB == 3)
            part[c] = (blk[0] + blk[1]) + blk[2];
        else if constexpr (NB == 2)
            part[c] = blk[0] + blk[1];
        else
            part[c] = blk[0];
    }
    float kk;
    if constexpr (NC == 4) {
        // lanes < 32 gather blocks 0 and 1, lanes >= 32 blocks 2 and 3 (the
        // upper half of one operand swapped with the lower half of the other);
        // then pairs of 16-lane rows leave row g with block g
        const auto h0 = __builtin_amdgcn_permlane32_swap(__float_as_uint(part[0]),
                                                         __float_as_uint(part[2]), false, false);
        const auto h1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(part[1]),
                                                         __float_as_uint(part[3]), false, false);
        const float k0 = __uint_as_float(h0[0]) + __uint_as_float(h0[1]);
        const float k1 = __uint_as_float(h1[0]) + __uint_as_float(h1[1]);
        const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(k0),
                                                          __float_as_uint(k1), false, false);
        kk = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
    } else {
        const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(part[0]),
                                                        __float_as_uint(part[1]), false, false);
        kk = __uint_as_float(h[0]) + __uint_as_float(h[1]);
        const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(kk),
                                                          __float_as_uint(kk), false, false);
        kk = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
    }
    float chi2 = kk * unscale;
    if constexpr (SCALED) chi2 = ldexpf(chi2, 2 * L.e_own);

    if (q == L.p_own) {
        L.cp = chi2;
        L.have_cp = true;
    }
    if (chi2 < L.best) {
        L.best = chi2;
        L.qbest = (uint32_t)q;
    }
    if (more) wait_record_loads();
    __syncthreads();
}

template <int CODE, int NC, bool FP16>
__device__ __forceinline__ void split_item(const ScanItem &it, uint4 *buf0, uint4 *buf1)
{
    static_assert(NC == 2 || NC == 4, "two or four 16-universe column blocks per wave");
    constexpr int SM = code_smax(CODE);
    constexpr int UW = 16 * NC;
    constexpr int REC = code_rec_units(CODE);
    constexpr int THREADS = 64 * kWavesPerBlock;
    static_assert(REC <= 5 * THREADS, "records of at most five 4 KB pieces");

    const uint4 *__restrict__ R16 = it.R;
    const double *__restrict__ d = it.d;
    const double *__restrict__ off = it.off;
    const int64_t K = it.K;
    const int N = it.N;
    const int ed = it.ed;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t u0 = it.u0 + wave * UW;
    const int64_t qb = it.qb, qe = it.qe;
    if (qb >= qe || K <= 0) return;  // uniform per block
    const int grp = lane >> 4, col = lane & 15;

    SplitLane<SM, NC> L;
    // the universes, split once: B operand of k-step s for column block c holds
    // positions p = 32s + 8*grp + e of universe u0 + 16c + col's k sequence,
    // i.e. bin j = p / 3 of 2^(ed - eu) (d - o), its low half where p % 3 = 1.
    // FP16: eu >= 0 is the universe's own power of two, 0 while its largest
    // |d - o| 2^ed is below 65504 (FP16's largest finite value: hi rounds to at
    // most that, lo is its small rest), i.e. for every universe within 8x the
    // grid's range of S - o (ed keeps that below 2^13), and the values are then
    // the grid-wide scale's; beyond, |d - o| 2^(ed - eu) lands in [2^14, 2^15).
    // eu is kept to 8 bits: a universe beyond 2^269 (whose chi^2 overflows FP32
    // anyway) saturates.
    bool any_scaled = false;
    L.eu_pk = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int64_t u = u0 + 16 * c + col;
        int eu = 0;
        if constexpr (FP16) {
            double m = 0.0;
            for (int k = 8 * grp; k < N; k += 32)
                for (int e = 0; e < 8; ++e)
                    if (u < K && k + e < N) m = fmax(m, fabs(d[u * N + k + e] - off[k + e]));
            m = ldexp(m, ed);
            m = fmax(m, __shfl_xor(m, 16));  // the universe's four lane rows
            m = fmax(m, __shfl_xor(m, 32));
            if (m >= 65504.0 && m <= 1.0e300) eu = min(ilogb(m) - 14, 255);
        }
        L.eu_pk |= (uint32_t)eu << (8 * c);
        any_scaled = any_scaled || eu != 0;
    }
    // a fragment's eight positions 32s + 8*grp + e cover at most four bins
    // from j0 = (32s + 8*grp) / 3: those are loaded (from clamped, in-range
    // addresses, the values then masked) and spread; one step at a time for
    // all column blocks, so that only that step's loads are in flight
#pragma unroll
    for (int s = 0; s < SM; ++s) {
        const int p0 = 32 * s + 8 * grp, j0 = p0 / 3, r0 = p0 - 3 * j0;
        double o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = off[j0 + i < N ? j0 + i : N - 1];
        uint32_t lomask = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) lomask |= ((r0 + e) % 3 == 1 ? 1u : 0u) << e;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int64_t u = u0 + 16 * c + col;
            const bool uin = u < K;
            const double *__restrict__ du = d + (uin ? u : K - 1) * (int64_t)N;
            const int sc = ed - (int)((L.eu_pk >> (8 * c)) & 255u);
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = j0 + i;
                const double dv = du[k < N ? k : N - 1] - o[i];
                v[i] = (uin && k < N) ? (float)ldexp(dv, sc) : 0.0f;
            }
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = (r0 + e) / 3;  // 0..3
                x[e] = i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
            }
            uint4 hi, lo;
            split8<FP16>(x, hi, lo);
            L.dx[c][s] = pick_lo(hi, lo, lomask);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    L.scaled = __any(any_scaled);
    // after the reduction, lane l holds column block cl of universe column col
    const int cl = (NC == 4) ? grp : (grp >> 1);
    const bool owner = (NC == 4) ? true : ((grp & 1) == 0);
    const int64_t u_own = u0 + 16 * cl + col;
    L.e_own = (int)((L.eu_pk >> (8 * cl)) & 255u);
    L.p_own = (u_own < K) ? (it.p_idx ? it.p_idx[u_own] : it.p) : -1;
    L.best = __builtin_inff();
    L.qbest = 0xffffffffu;
    L.cp = 0.0f;
    L.have_cp = false;

    record_to_lds<REC, THREADS>(R16 + qb * REC, buf0, tid);
    wait_record_loads();
    __syncthreads();
    // a wave with a universe outside the FP16 range runs the loop that
    // rescales its accumulators; every other wave runs the plain one
    int64_t q = qb;
    if (FP16 && L.scaled) {
        for (; q + 1 < qe; q += 2) {
            split_point<CODE, NC, FP16, FP16>(q, true, R16, buf0, buf1, L);
            split_point<CODE, NC, FP16, FP16>(q + 1, q + 2 < qe, R16, buf1, buf0, L);
        }
        if (q < qe) split_point<CODE, NC, FP16, FP16>(q, false, R16, buf0, buf1, L);
    } else {
        for (; q + 1 < qe; q += 2) {
            split_point<CODE, NC, FP16, false>(q, true, R16, buf0, buf1, L);
            split_point<CODE, NC, FP16, false>(q + 1, q + 2 < qe, R16, buf1, buf0, L);
        }
        if (q < qe) split_point<CODE, NC, FP16, false>(q, false, R16, buf0, buf1, L);
    }

    if (owner && u_own < K) {
        if (L.have_cp) it.chi2_p[u_own] = (double)L.cp;
        if (L.best < __builtin_inff()) {
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(L.best) << 32) | (unsigned long long)L.qbest;
            atomicMin(&it.keys[u_own], key);
        }
    }
}

// Waves per SIMD the kernel is built for: three while the B fragments and
// the accumulators (4 NC (smax + nb) VGPRs) leave room for the rest in a
// third of the register file, else two.
template <int CODE, int NC>
constexpr int split_waves()
{
    return 4 * NC * (code_smax(CODE) + code_nb(CODE)) + 40 <= 168 ? 3 : 2;
}

template <int CODE, int NC, bool FP16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(split_waves<CODE, NC>())))
void k_scan_split(const uint4 *__restrict__ R16, const double *__restrict__ d,
                  const double *__restrict__ off, int ed, const int64_t *__restrict__ p_idx,
                  int64_t K, int N, int64_t q_lo, int64_t q_hi, int64_t n_utiles,
                  int64_t q_per_chunk, unsigned long long *__restrict__ keys,
                  double *__restrict__ chi2_p)
{
    __shared__ uint4 buf0[code_rec_units(CODE)], buf1[code_rec_units(CODE)];
    ScanItem it;
    it.R = R16;
    it.d = d;
    it.p_idx = p_idx;
    it.p = -1;
    it.keys = keys;
    it.chi2_p = chi2_p;
    it.off = off;
    it.K = K;
    it.N = N;
    it.ed = ed;
    const int64_t utile = blockIdx.x % n_utiles;
    const int64_t qchunk = blockIdx.x / n_utiles;
    it.u0 = utile * (int64_t)(16 * NC * kWavesPerBlock);
    it.qb = q_lo + qchunk * q_per_chunk;
    it.qe = (it.qb + q_per_chunk < q_hi) ? it.qb + q_per_chunk : q_hi;
    split_item<CODE, NC, FP16>(it, buf0, buf1);
}

// Serving: persistent-style launch over a finite table of items (see the
// FP32 form).
template <int CODE, int NC, bool FP16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_serve_split(
    const ScanItem *__restrict__ items, int n_items, int *__restrict__ counter)
{
    __shared__ uint4 buf0[code_rec_units(CODE)], buf1[code_rec_units(CODE)];
    __shared__ int cur;
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
        __syncthreads();
        const int i = cur;
        __syncthreads();
        if (i >= n_items) break;
        split_item<CODE, NC, FP16>(items[i], buf0, buf1);
        __syncthreads();
    }
}

static int resident_slots_split(const void *kernel)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 512;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 2;
    return cus * per_cu;
}

constexpr int kSplitColBlocks = 4;  // 64 universes per wave
// Grid points per block at most.  The blocks that share a chunk read the
// same records in the same order, and the L2 serves the later readers only
// while the blocks stay within a few hundred points of each other; short
// chunks restart them together often (c5, 2048 instead of 25 600 points:
// split FP16 7.6 -> 5.6 TB fetched, 1.82 -> 1.66 s; BF16 3.3 -> 1.2 TB).
constexpr int64_t kSplitChunkMax = 2048;

// Every layout split_code gives for N = 1..64 (step counts of the row groups).
#define FC_SPLIT_CODES(X)                                                                   \
    X(0x0001) X(0x0002) X(0x0021) X(0x0031) X(0x0032) X(0x0421) X(0x0431) X(0x0532)        \
        X(0x5421) X(0x6431) X(0x6532)

constexpr bool split_code_known(int code)
{
#define FC_K(c) if (code == (c)) return true;
    FC_SPLIT_CODES(FC_K)
#undef FC_K
    return false;
}
constexpr bool split_codes_cover(int n)
{
    return n > 64 || (split_code_known(split_code(n)) && split_codes_cover(n + 1));
}
static_assert(split_codes_cover(1), "a bin count without a split-form kernel");

template <int CODE, bool FP16>
static hipError_t launch_split_t(const fc_grid *g, int64_t K, const double *d,
                                 const int64_t *p_idx, int64_t q0, int64_t nq,
                                 unsigned long long *keys, double *chi2_p, hipStream_t st)
{
    constexpr int NC = kSplitColBlocks;
    // resident block slots: queried once per instantiation (thread-safe)
    static const int slots =
        resident_slots_split(reinterpret_cast<const void *>(&k_scan_split<CODE, NC, FP16>));
    ScanGeometry sg = scan_geometry(K, nq, slots, 16 * NC * kWavesPerBlock);
    if (sg.q_per_chunk > kSplitChunkMax) {
        // shorter chunks, as many as keep blocks x 256 work-items within the
        // 32-bit dispatch size (the general geometry's bound)
        const int64_t cap = (int64_t(1) << 23) / (sg.n_utiles > 0 ? sg.n_utiles : 1);
        int64_t nc = (nq + kSplitChunkMax - 1) / kSplitChunkMax;
        if (nc > cap) nc = cap;
        if (nc > sg.n_qchunks) {
            sg.q_per_chunk = (nq + nc - 1) / nc;
            sg.n_qchunks = (nq + sg.q_per_chunk - 1) / sg.q_per_chunk;
        }
    }
    const int64_t blocks = sg.n_utiles * sg.n_qchunks;
    const uint4 *R = FP16 ? g->RH16 : g->RB16;
    ProfScope prof(st, "k_scan_split");
    hipLaunchKernelGGL((k_scan_split<CODE, NC, FP16>), dim3((unsigned)blocks), dim3(256), 0, st,
                       R, d, g->off, FP16 ? g->ed16 : 0, p_idx, K, g->N, q0, q0 + nq,
                       sg.n_utiles, sg.q_per_chunk, keys, chi2_p);
    return hipGetLastError();
}

template <int CODE, bool FP16>
static int serve_slots_split_t()
{
    // resident block slots: queried once per instantiation (thread-safe)
    static const int slots = resident_slots_split(
        reinterpret_cast<const void *>(&k_serve_split<CODE, kSplitColBlocks, FP16>));
    return slots;
}

template <int CODE, bool FP16>
static hipError_t launch_serve_split_t(const ScanItem *items, int n_items, int *counter,
                                       int blocks, hipStream_t st)
{
    hipLaunchKernelGGL((k_serve_split<CODE, kSplitColBlocks, FP16>), dim3((unsigned)blocks),
                       dim3(256), 0, st, items, n_items, counter);
    return hipGetLastError();
}

int serve_split_univ_per_item() { return 16 * kSplitColBlocks * kWavesPerBlock; }

hipError_t launch_serve_split(int code, bool fp16, const ScanItem *items, int n_items,
                              int *counter, int blocks, hipStream_t st)
{
#define FC_CASE_T(c) \
    case c: return launch_serve_split_t<c, true>(items, n_items, counter, blocks, st);
#define FC_CASE_F(c) \
    case c: return launch_serve_split_t<c, false>(items, n_items, counter, blocks, st);
    if (fp16) {
        switch (code) { FC_SPLIT_CODES(FC_CASE_T) }
    } else {
        switch (code) { FC_SPLIT_CODES(FC_CASE_F) }
    }
#undef FC_CASE_T
#undef FC_CASE_F
    return hipErrorInvalidValue;
}

int serve_slots_split(int code, bool fp16)
{
#define FC_CASE_T(c) \
    case c: return serve_slots_split_t<c, true>();
#define FC_CASE_F(c) \
    case c: return serve_slots_split_t<c, false>();
    if (fp16) {
        switch (code) { FC_SPLIT_CODES(FC_CASE_T) }
    } else {
        switch (code) { FC_SPLIT_CODES(FC_CASE_F) }
    }
#undef FC_CASE_T
#undef FC_CASE_F
    return 512;
}

hipError_t launch_scan_split(const fc_grid *g, bool fp16, int64_t K, const double *d,
                             const int64_t *p_idx, int64_t q0, int64_t nq,
                             unsigned long long *keys, double *chi2_p, hipStream_t st)
{
    const int code = split_code(g->N);
#define FC_CASE_T(c) \
    case c: return launch_split_t<c, true>(g, K, d, p_idx, q0, nq, keys, chi2_p, st);
#define FC_CASE_F(c) \
    case c: return launch_split_t<c, false>(g, K, d, p_idx, q0, nq, keys, chi2_p, st);
    if (fp16) {
        switch (code) { FC_SPLIT_CODES(FC_CASE_T) }
    } else {
        switch (code) { FC_SPLIT_CODES(FC_CASE_F) }
    }
#undef FC_CASE_T
#undef FC_CASE_F
    return hipErrorInvalidValue;
}

}  // namespace fcx
