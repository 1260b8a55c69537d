// k_scan.hip -- the chi^2 grid scan (Eq. (1) inside Algorithm 1's loops).
//
// FP32 form (the hot kernel).  Eq. (1) is evaluated in factor form,
//     chi2(d, q) = ||W_q (d - S_q)||^2,   W_q = L_q^{-1} (lower triangular),
// which equals (d-S_q)^T Sigma_q^{-1} (d-S_q).  For a fixed q and a tile of
// universes this is a dense contraction Z = W_q R (R = bins x universes),
// done on the matrix cores with v_mfma_f32_16x16x4_f32 over the lower-
// triangular block pattern of W_q only, followed by a column-wise sum of
// squares, a reduction across the four 16-lane groups and a strict-"<"
// running minimum per universe.  Vector instructions do not overlap the FP32
// MFMAs on this chip, so the vector work around them (residuals, squares) is
// kept to few FP32 instructions: FP64 ones cost twice as much.
//
// Work decomposition: a 256-thread block owns a tile of 4 waves x 32
// universes and walks a contiguous range of grid points in list order.  Each
// wave keeps its universes' residual operands in registers; the block
// double-buffers one record per grid point in LDS (W_q fragments, S_q and the
// correction C_q), bringing the next record in with direct global -> LDS
// loads while the waves contract the current one, with one barrier per grid
// point.  Ranges of the same universes are merged with a
// 64-bit atomicMin on keys (FP32 chi2 bits above q), which reproduces
// Algorithm 1's rule that the lowest q wins exact ties whatever the split.
#include "fc_internal.h"

namespace fcx {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float pick(const float4 &v, int c)
{
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}

// Per grid point the block stages one record in LDS: the W_q fragments (NG
// groups of 1 KB), the FP32 part of S_q in B-operand order (256 B) and the
// correction C_q = -W_q (S_q - float(S_q)) in accumulator order (256 B).  Records are
// double-buffered: while the waves contract grid point q from one buffer, the
// block's 256 threads copy record q+1 into the other with coalesced 16-byte
// loads, and one barrier per grid point hands the buffers over.
template <int NS>
struct Fp32Geo {
    static constexpr int NB = n_rowblocks_from_ns(NS);
    static constexpr int NG = n_groups_from_ns(NS);
    static constexpr int NWU = rec_w_units(NS);  // 16-byte units of W per record
    static constexpr int REC = rec_units(NS);    // W + 512 B of S and C
};

// Per-universe state a wave carries through its range of grid points.
template <int NS, int NC>
struct Fp32Lane {
    float dh[NC][NS], dl[NC][NS];  // B-operand sources d = dh + dl
    int64_t p_own;                 // true point of the universe this lane reports
    float best;                    // running minimum and its grid point
    uint32_t qbest;
    float cp;                      // chi2 at the true point, once seen
    bool have_cp;
};

// One grid point: contract the record in `cur`, fold chi2 into the running
// minimum, and (if more) bring the next record into `nxt`.  The two LDS
// buffers are separate objects so that the compiler can tell the copy into
// one from the reads of the other.
template <int NS, int NC>
__device__ __forceinline__ void fp32_point(int64_t q, bool more, const uint4 *__restrict__ R32,
                                           const uint4 *cur, uint4 *nxt, Fp32Lane<NS, NC> &L)
{
    constexpr int NB = Fp32Geo<NS>::NB;
    constexpr int NWU = rec_w_units(NS);
    constexpr int REC = rec_units(NS);
    constexpr int THREADS = 64 * kWavesPerBlock;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int grp = lane >> 4;

    if (more) record_to_lds<REC, THREADS>(R32 + (q + 1) * REC, nxt, tid);
    __builtin_amdgcn_sched_barrier(0);  // issue the copy before the contraction

    const float4 *wl = reinterpret_cast<const float4 *>(cur);
    const float *shl = reinterpret_cast<const float *>(cur + NWU) + grp * 16;
    // accumulators start at C_q: rows 4 grp .. 4 grp + 3 of each row block
    const float4 *cl = reinterpret_cast<const float4 *>(cur + NWU) + 16 + grp;
    v4f acc[NC][NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const float4 cv = cl[4 * b];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c][b] = v4f{cv.x, cv.y, cv.z, cv.w};
    }

    float4 wv = wl[lane];
    int wg_loaded = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const float sh = shl[s];
        float r[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] = (L.dh[c][s] - sh) + L.dl[c][s];
#pragma unroll
        for (int b = first_block_of_kstep(NS, s); b < NB; ++b) {
            const int t = pair_index(NS, s, b);
            if ((t >> 2) != wg_loaded) {
                wg_loaded = t >> 2;
                wv = wl[wg_loaded * 64 + lane];
            }
            const float w = pick(wv, t & 3);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                acc[c][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, r[c], acc[c][b], 0, 0, 0);
        }
    }

    // sum of squares per universe column: FP32 chains of the 4 rows a lane
    // holds per row block, a pairwise tree over the blocks, then the four
    // lane groups (FP32 instructions only)
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
        // reduce-scatter: lane l ends with column block l/16
        const bool hi = lane >= 32;
        float k0 = hi ? part[2] : part[0];
        float k1 = hi ? part[3] : part[1];
        const float s0 = hi ? part[0] : part[2];
        const float s1 = hi ? part[1] : part[3];
        k0 += __shfl_xor(s0, 32);
        k1 += __shfl_xor(s1, 32);
        const bool odd = grp & 1;
        kk = odd ? k1 : k0;
        const float ss = odd ? k0 : k1;
        kk += __shfl_xor(ss, 16);
    } else {
        // lanes < 32 end with block 0, lanes >= 32 with block 1: swapping the
        // upper half of part[0] with the lower half of part[1] leaves lane l
        // both halves of its block; then rows of 16 lanes are paired
        const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(part[0]),
                                                        __float_as_uint(part[1]), false, false);
        kk = __uint_as_float(h[0]) + __uint_as_float(h[1]);
        const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(kk),
                                                          __float_as_uint(kk), false, false);
        kk = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
    }
    const float chi2 = kk;

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

template <int NS, int NC>
__device__ __forceinline__ void fp32_item(const ScanItem &it, uint4 *buf0, uint4 *buf1)
{
    static_assert(NC == 2 || NC == 4, "two or four 16-universe column blocks per wave");
    constexpr int NG = Fp32Geo<NS>::NG;
    constexpr int UW = 16 * NC;            // universes per wave
    constexpr int NWU = rec_w_units(NS);   // 16-byte units of W per record
    constexpr int REC = rec_units(NS);     // W + 512 B of S and C
    constexpr int THREADS = 64 * kWavesPerBlock;
    static_assert(REC <= 3 * THREADS, "records of at most three 4 KB pieces");
    static_assert(NG * 64 == NWU, "W groups");

    const uint4 *__restrict__ R32 = it.R;
    const double *__restrict__ d = it.d;
    const int64_t K = it.K;
    const int N = it.N;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t u0 = it.u0 + wave * UW;
    const int64_t qb = it.qb, qe = it.qe;
    if (qb >= qe) return;  // uniform per block
    const int grp = lane >> 4, col = lane & 15;

    Fp32Lane<NS, NC> L;
    // B-operand sources as FP32 pairs d = dh + dl: universe u0+16c+col, bin
    // 4s+grp (zero past N and past K; waves past K still take part in the
    // copies and barriers)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int64_t u = u0 + 16 * c + col;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = 4 * s + grp;
            const double v = (u < K && k < N) ? d[u * N + k] : 0.0;
            L.dh[c][s] = (float)v;
            L.dl[c][s] = (float)(v - (double)L.dh[c][s]);
        }
    }
    // after the reduction, lane l holds column block cl of universe column col
    const int cl = (NC == 4) ? grp : (grp >> 1);
    const bool owner = (NC == 4) ? true : ((grp & 1) == 0);
    const int64_t u_own = u0 + 16 * cl + col;
    L.p_own = (u_own < K) ? (it.p_idx ? it.p_idx[u_own] : it.p) : -1;
    L.best = __builtin_inff();
    L.qbest = 0xffffffffu;
    L.cp = 0.0f;
    L.have_cp = false;

    record_to_lds<REC, THREADS>(R32 + qb * REC, buf0, tid);
    wait_record_loads();
    __syncthreads();
    // grid points in pairs so that each one's LDS buffer is fixed
    int64_t q = qb;
    for (; q + 1 < qe; q += 2) {
        fp32_point<NS, NC>(q, true, R32, buf0, buf1, L);
        fp32_point<NS, NC>(q + 1, q + 2 < qe, R32, buf1, buf0, L);
    }
    if (q < qe) fp32_point<NS, NC>(q, false, R32, buf0, buf1, L);

    if (owner && u_own < K) {
        if (L.have_cp) it.chi2_p[u_own] = (double)L.cp;
        if (L.best < __builtin_inff()) {
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(L.best) << 32) | (unsigned long long)L.qbest;
            atomicMin(&it.keys[u_own], key);
        }
    }
}

template <int NS, int NC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_scan_fp32(
    const uint4 *__restrict__ R32, const double *__restrict__ d,
    const int64_t *__restrict__ p_idx, int64_t K, int N, int64_t G, int64_t n_utiles,
    int64_t q_per_chunk, unsigned long long *__restrict__ keys, double *__restrict__ chi2_p)
{
    __shared__ uint4 buf0[Fp32Geo<NS>::REC], buf1[Fp32Geo<NS>::REC];
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
    it.u0 = utile * (int64_t)(16 * NC * kWavesPerBlock);
    it.qb = qchunk * q_per_chunk;
    it.qe = (it.qb + q_per_chunk < G) ? it.qb + q_per_chunk : G;
    fp32_item<NS, NC>(it, buf0, buf1);
}

// Serving: a persistent-style launch over a table of items (any mix of
// requests and grids with this bin count).  Resident blocks take items in
// turn from an atomic counter until the table is exhausted; the table is
// finite and fixed at launch, so every block reaches the exit.
template <int NS, int NC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_serve_fp32(
    const ScanItem *__restrict__ items, int n_items, int *__restrict__ counter)
{
    __shared__ uint4 buf0[Fp32Geo<NS>::REC], buf1[Fp32Geo<NS>::REC];
    __shared__ int cur;
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
        __syncthreads();
        const int i = cur;
        __syncthreads();
        if (i >= n_items) break;
        fp32_item<NS, NC>(items[i], buf0, buf1);
        __syncthreads();
    }
}

// FP64 form: one thread per universe over the whole grid (the parity anchor).
// W_q is uniform across the wave, so its entries arrive through scalar loads.
template <int NP>
__global__ __launch_bounds__(64) void k_scan_fp64(
    const double *__restrict__ W64, const double *__restrict__ S64, const double *__restrict__ d,
    const int64_t *__restrict__ p_idx, int64_t K, int N, int64_t G, double *__restrict__ dchi2,
    double *__restrict__ chi2_min, int64_t *__restrict__ argmin, double *__restrict__ chi2_p)
{
    const int64_t u = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (u >= K) return;
    const int64_t NT = (int64_t)N * (N + 1) / 2;
    double dv[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) dv[j] = (j < N) ? d[u * N + j] : 0.0;
    const int64_t p = p_idx[u];
    double best = __builtin_inf();
    int64_t qbest = p;
    double cp = __builtin_nan("");
    for (int64_t q = 0; q < G; ++q) {
        const double *Wq = W64 + q * NT;
        const double *Sq = S64 + q * N;
        double r[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) r[j] = (j < N) ? dv[j] - Sq[j] : 0.0;
        double chi2 = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (i < N) {
                double z = 0.0;
#pragma unroll
                for (int j = 0; j <= i; ++j) z = fma(Wq[tri_index(i, j)], r[j], z);
                chi2 = fma(z, z, chi2);
            }
        }
        if (q == p) cp = chi2;
        if (chi2 < best) {
            best = chi2;
            qbest = q;
        }
    }
    chi2_min[u] = best;
    argmin[u] = qbest;
    chi2_p[u] = cp;
    dchi2[u] = cp - best;
}

__global__ __launch_bounds__(256) void k_init_keys(int64_t K, unsigned long long *__restrict__ keys,
                                                  double *__restrict__ chi2_p)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= K) return;
    keys[u] = kKeyNone;
    chi2_p[u] = __builtin_nan("");
}

// Decode the keys in place (the key buffer is the caller's chi2_min array).
__global__ __launch_bounds__(256) void k_finalize(int64_t K, const int64_t *__restrict__ p_idx,
                                                 int64_t p_uniform,
                                                 unsigned long long *__restrict__ keys,
                                                 int64_t *__restrict__ argmin,
                                                 const double *__restrict__ chi2_p,
                                                 double *__restrict__ dchi2)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= K) return;
    const unsigned long long key = keys[u];
    const uint32_t hi = (uint32_t)(key >> 32);
    double cmin;
    int64_t am;
    if (hi >= 0x7f800000u) {  // no chi2 < +inf was seen: Algorithm 1's initial state
        cmin = __builtin_inf();
        am = p_idx ? p_idx[u] : p_uniform;
    } else {
        cmin = (double)__uint_as_float(hi);
        am = (int64_t)(uint32_t)(key & 0xffffffffu);
    }
    reinterpret_cast<double *>(keys)[u] = cmin;
    argmin[u] = am;
    dchi2[u] = chi2_p[u] - cmin;
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
// block slots with the smallest tail: minimise ceil(tiles*c/slots)/c.
ScanGeometry scan_geometry(int64_t K, int64_t G, int slots, int univ_per_block)
{
    ScanGeometry sg;
    sg.n_utiles = (K + univ_per_block - 1) / univ_per_block;
    const int64_t min_chunk = 64;
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

template <int NS>
static hipError_t launch_fp32_ns(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                                 unsigned long long *keys, double *chi2_p, hipStream_t st)
{
    constexpr int NC = kScanColBlocks;
    static int slots = 0;  // per instantiation; same device model for the process
    if (slots == 0)
        slots = resident_slots(reinterpret_cast<const void *>(&k_scan_fp32<NS, NC>),
                               64 * kWavesPerBlock);
    const ScanGeometry sg = scan_geometry(K, g->G, slots, 16 * NC * kWavesPerBlock);
    const int64_t blocks = sg.n_utiles * sg.n_qchunks;
    hipLaunchKernelGGL((k_scan_fp32<NS, NC>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0,
                       st, g->R32, d, p_idx, K, g->N, g->G, sg.n_utiles, sg.q_per_chunk, keys,
                       chi2_p);
    return hipGetLastError();
}

template <int NS>
static hipError_t launch_serve_fp32_ns(const ScanItem *items, int n_items, int *counter, int blocks,
                                       hipStream_t st)
{
    hipLaunchKernelGGL((k_serve_fp32<NS, kScanColBlocks>), dim3((unsigned)blocks), dim3(256), 0, st,
                       items, n_items, counter);
    return hipGetLastError();
}

template <int NS>
static int serve_slots_fp32_ns()
{
    static int slots = 0;
    if (slots == 0)
        slots = resident_slots(reinterpret_cast<const void *>(&k_serve_fp32<NS, kScanColBlocks>), 256);
    return slots;
}

int serve_fp32_univ_per_item() { return 16 * kScanColBlocks * kWavesPerBlock; }

hipError_t launch_serve_fp32(int ns, const ScanItem *items, int n_items, int *counter, int blocks,
                             hipStream_t st)
{
    switch (ns) {
#define FC_CASE(n) \
    case n: return launch_serve_fp32_ns<n>(items, n_items, counter, blocks, st);
        FC_CASE(1) FC_CASE(2) FC_CASE(3) FC_CASE(4) FC_CASE(5) FC_CASE(6) FC_CASE(7) FC_CASE(8)
        FC_CASE(9) FC_CASE(10) FC_CASE(11) FC_CASE(12) FC_CASE(13) FC_CASE(14) FC_CASE(15)
        FC_CASE(16)
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

int serve_slots_fp32(int ns)
{
    switch (ns) {
#define FC_CASE(n) \
    case n: return serve_slots_fp32_ns<n>();
        FC_CASE(1) FC_CASE(2) FC_CASE(3) FC_CASE(4) FC_CASE(5) FC_CASE(6) FC_CASE(7) FC_CASE(8)
        FC_CASE(9) FC_CASE(10) FC_CASE(11) FC_CASE(12) FC_CASE(13) FC_CASE(14) FC_CASE(15)
        FC_CASE(16)
#undef FC_CASE
    default: return 512;
    }
}

hipError_t launch_scan_fp32(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                            unsigned long long *keys, double *chi2_p, hipStream_t st)
{
    switch (g->ns) {
#define FC_CASE(n) \
    case n: return launch_fp32_ns<n>(g, K, d, p_idx, keys, chi2_p, st);
        FC_CASE(1) FC_CASE(2) FC_CASE(3) FC_CASE(4) FC_CASE(5) FC_CASE(6) FC_CASE(7) FC_CASE(8)
        FC_CASE(9) FC_CASE(10) FC_CASE(11) FC_CASE(12) FC_CASE(13) FC_CASE(14) FC_CASE(15)
        FC_CASE(16)
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

template <int NP>
static hipError_t launch_fp64_np(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                                 double *dchi2, double *chi2_min, int64_t *argmin, double *chi2_p,
                                 hipStream_t st)
{
    const int64_t blocks = (K + 63) / 64;
    hipLaunchKernelGGL(k_scan_fp64<NP>, dim3((unsigned)blocks), dim3(64), 0, st, g->W64, g->S64, d,
                       p_idx, K, g->N, g->G, dchi2, chi2_min, argmin, chi2_p);
    return hipGetLastError();
}

hipError_t launch_scan_fp64(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                            double *dchi2, double *chi2_min, int64_t *argmin, double *chi2_p,
                            hipStream_t st)
{
    const int np = ((g->N + 7) / 8) * 8;
    switch (np) {
#define FC_CASE(n) \
    case n: return launch_fp64_np<n>(g, K, d, p_idx, dchi2, chi2_min, argmin, chi2_p, st);
        FC_CASE(8) FC_CASE(16) FC_CASE(24) FC_CASE(32) FC_CASE(40) FC_CASE(48) FC_CASE(56)
        FC_CASE(64)
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init_keys(int64_t K, unsigned long long *keys, double *chi2_p, hipStream_t st)
{
    const int64_t blocks = (K + 255) / 256;
    hipLaunchKernelGGL(k_init_keys, dim3((unsigned)blocks), dim3(256), 0, st, K, keys, chi2_p);
    return hipGetLastError();
}

hipError_t launch_finalize(int64_t K, const int64_t *p_idx, unsigned long long *keys_as_chi2_min,
                           int64_t *argmin, const double *chi2_p, double *dchi2, hipStream_t st,
                           int64_t p_uniform)
{
    const int64_t blocks = (K + 255) / 256;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)blocks), dim3(256), 0, st, K, p_idx, p_uniform,
                       keys_as_chi2_min, argmin, chi2_p, dchi2);
    return hipGetLastError();
}

}  // namespace fcx
