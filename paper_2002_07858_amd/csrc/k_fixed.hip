// k_fixed.hip -- Algorithm 1 with one matrix for the whole grid, and the
// iteration of that matrix (Section 2, step 5).
//
// Algorithm 1 as printed passes a single M to every chi^2 of a universe's
// scan.  With M = Sigma_m^{-1} = W_m^T W_m (W_m = L_m^{-1}, the FP64 factor
// of grid point m) and a per-bin offset o,
//     chi2(d, q) = ||y - t_q||^2 = a + b_q - 2 y.t_q,
//     y = W_m (d - o),  a = ||y||^2,  t_q = W_m (S_q - o),  b_q = ||t_q||^2,
// so one universe tile against all grid points is a dense GEMM (universes x
// bins) . (bins x grid points) with an epilogue that forms chi2 and keeps the
// running minimum -- the same contraction as a nearest-neighbour search in
// the space whitened by W_m.  It runs on v_mfma_f64_16x16x4_f64 in FP64:
// a + b - 2 y.t cancels a factor ~(a + b)/chi2 (about 1e2 here), which FP64
// absorbs with room to spare (error ~1e-13 relative to chi2).
//
// m starts at the universe's true point p.  For the iterated variant, after a
// scan whose minimiser q_min differs from m the universe is scanned again
// with m = q_min, until q_min repeats or an iteration cap.  Universes are
// grouped by m on the host (counting sort); each group's t_q are built once
// per round.
//
// GEMM kernel: a 256-thread block owns 64 universes of one group (4 column
// blocks of 16) and a chunk of grid points; each wave contracts 16 grid
// points per step against the block's universes, whose y fragments stay in
// registers; the t tile (64 points x 4*NS bins) is double-buffered in LDS and
// brought in by direct global -> LDS loads while the previous tile is used.
// Per-chunk minima (value, q) are merged by a small kernel with Algorithm 1's
// rule (smallest value, then lowest q).
#include "fc_internal.h"

#include <algorithm>
#include <vector>

namespace fcx {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kFxTile = 64;      // universes per block, grid points per step
constexpr int kFxThreads = 256;

// y = W_m (d - o), a = ||y||^2 for universe rows in group order: one wave per
// row, lane i = component i (zero past N, stored padded to 4 * ns).
__global__ __launch_bounds__(256) void k_fixed_y(const double *__restrict__ W64,
                                                 const double *__restrict__ d,
                                                 const double *__restrict__ off,
                                                 const int64_t *__restrict__ order,
                                                 const int64_t *__restrict__ m_of_row, int N,
                                                 int np, int64_t R, double *__restrict__ Y,
                                                 double *__restrict__ a)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= R) return;  // whole wave
    const int64_t k = order[r];
    const double *Wm = W64 + m_of_row[r] * ((int64_t)N * (N + 1) / 2);
    const double x = (lane < N) ? d[k * N + lane] - off[lane] : 0.0;
    double y = 0.0;
    const int row = lane < N ? lane : 0;
    for (int j = 0; j < N; ++j) {
        const double xj = __shfl(x, j);
        if (j <= row) y = fma(Wm[(int64_t)row * (row + 1) / 2 + j], xj, y);
    }
    if (lane >= N) y = 0.0;
    if (lane < np) Y[r * np + lane] = y;
    double s = y * y;
    for (int w = 32; w > 0; w >>= 1) s += __shfl_xor(s, w);
    if (lane == 0) a[r] = s;
}

// t_q = W_m (S_q - o), b_q = ||t_q||^2 for 64 grid points q of matrix slot ms
// per block, on the FP64 matrix cores: wave w forms rows q0 + 16w .. +15 of
// T = X W^T (X = signal rows minus the offset), four 16-column blocks of
// components, k-steps of four bins; W^T comes from LDS (zero above the
// diagonal and past N), X straight from the signal table.
template <int NS>
__global__ __launch_bounds__(256) void k_fixed_t(const double *__restrict__ W64,
                                                 const double *__restrict__ S64,
                                                 const double *__restrict__ off,
                                                 const int64_t *__restrict__ m_of_slot, int N,
                                                 int64_t G, int64_t n_qtiles, int64_t b_stride,
                                                 double *__restrict__ T, double *__restrict__ b)
{
    constexpr int NP = 4 * NS;
    constexpr int NC = (NP + 15) / 16;     // 16-column blocks of components
    __shared__ double wt[NP * 16 * NC];    // wt[j][i] = W_m[i][j]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 4, col = lane & 15;
    const int64_t ms = blockIdx.x / n_qtiles;
    const int64_t q0 = (blockIdx.x % n_qtiles) * 64;
    const double *Wm = W64 + m_of_slot[ms] * ((int64_t)N * (N + 1) / 2);
    for (int e = tid; e < NP * 16 * NC; e += 256) {
        const int j = e / (16 * NC), i = e % (16 * NC);
        wt[e] = (i < N && j <= i) ? Wm[(int64_t)i * (i + 1) / 2 + j] : 0.0;
    }
    __syncthreads();
    // A operand: row q = q0 + 16 wave + col, bins 4s + grp
    const int64_t qa = q0 + 16 * wave + col;
    const bool qa_in = qa < G;
    v4d acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int j = 4 * s + grp;
        const double x = (qa_in && j < N) ? S64[qa * N + j] - off[j] : 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, wt[j * 16 * NC + 16 * c + col], acc[c],
                                                          0, 0, 0);
    }
    // FP64 output layout: register r holds row grp + 4 r, column col of block c
    double *Tm = T + ms * G * NP;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t q = q0 + 16 * wave + grp + 4 * r;
        double sq = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int i = 16 * c + col;
            const double t = acc[c][r];
            if (q < G && i < NP) Tm[q * NP + i] = t;
            sq = fma(t, t, sq);   // components past N are exactly zero
        }
        for (int w = 1; w < 16; w <<= 1) sq += __shfl_xor(sq, w);
        if (col == 0 && q < G) b[ms * b_stride + q] = sq;
    }
}

struct FxTileDesc {
    int64_t r0;     // first row (group order) of the tile
    int32_t n;      // rows in the tile (1..64)
    int32_t slot;   // matrix slot of the group
};

// Running minimum of one (tile, grid chunk): candidates cand_v/cand_q
// [row][n_chunks], chi2 at the true point into cp[row] (exactly one block
// meets q == p for each row).
template <int NS>
__global__ __launch_bounds__(kFxThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_fixed_min(
    const FxTileDesc *__restrict__ tiles, int64_t n_tiles, const double *__restrict__ Y,
    const double *__restrict__ a, const int64_t *__restrict__ p_of_row,
    const double *__restrict__ T, const double *__restrict__ b, int64_t b_stride, int64_t G,
    int64_t q_per_chunk, int n_chunks, double *__restrict__ cand_v, int64_t *__restrict__ cand_q,
    double *__restrict__ cp)
{
    constexpr int NP = 4 * NS;             // padded bins
    constexpr int TU = kFxTile * NP / 2;   // 16-byte units of a t tile (rows contiguous)
    constexpr int TC = (TU + kFxThreads - 1) / kFxThreads;
    __shared__ uint4 t0[TC * kFxThreads], t1[TC * kFxThreads];
    __shared__ uint4 b0[kFxTile / 2], b1[kFxTile / 2];
    __shared__ double red_v[4][kFxTile];
    __shared__ int32_t red_q[4][kFxTile];

    const int64_t tile = blockIdx.x % n_tiles;
    const int chunk = (int)(blockIdx.x / n_tiles);
    const FxTileDesc td = tiles[tile];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 4, col = lane & 15;
    const int64_t qb = (int64_t)chunk * q_per_chunk;
    const int64_t qe = (qb + q_per_chunk < G) ? qb + q_per_chunk : G;
    const double *Tm = T + (int64_t)td.slot * G * NP;
    const double *bm = b + (int64_t)td.slot * b_stride;  // 16-byte aligned rows

    // B operand: y of universe column 16c + col, bins 4s + grp (rows past the
    // tile read as zero and are never reported)
    double yf[4][NS];
    double av[4];
    int32_t pv[4];   // grid indices fit 31 bits (checked on the host)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int u = 16 * c + col;
        const bool in = u < td.n;
        const int64_t r = td.r0 + u;
#pragma unroll
        for (int s = 0; s < NS; ++s) yf[c][s] = in ? Y[r * NP + 4 * s + grp] : 0.0;
        av[c] = in ? a[r] : 0.0;
        pv[c] = in ? (int32_t)p_of_row[r] : -1;
    }
    double best[4], cpv[4];
    int32_t bq[4];
    bool hasp[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        best[c] = __builtin_inf();
        bq[c] = INT32_MAX;
        cpv[c] = 0.0;
        hasp[c] = false;
    }

    // the t tile of grid points q0 .. q0+63 (and their b) into LDS with
    // direct global -> LDS loads; rows at or past qe are not loaded (their
    // LDS rows hold stale values, and their results are never used)
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
    auto stage = [&](uint4 *tdst, uint4 *bdst, int64_t q0) {
        const uint4 *src = reinterpret_cast<const uint4 *>(Tm + q0 * NP);
        if (q0 + kFxTile <= qe) {  // uniform: a whole tile, no per-row check
#pragma unroll
            for (int c = 0; c < TC; ++c) {
                const int unit = c * kFxThreads + tid;
                if (unit < TU)
                    __builtin_amdgcn_global_load_lds(
                        (const void *)(src + unit),
                        (__attribute__((address_space(3))) void *)(tdst + c * kFxThreads + wbase),
                        16, 0, 0);
            }
        } else {
#pragma unroll
            for (int c = 0; c < TC; ++c) {
                const int unit = c * kFxThreads + tid;
                if (unit < TU && q0 + unit / (NP / 2) < qe)
                    __builtin_amdgcn_global_load_lds(
                        (const void *)(src + unit),
                        (__attribute__((address_space(3))) void *)(tdst + c * kFxThreads + wbase),
                        16, 0, 0);
            }
        }
        // b in pairs of rows (rows are padded so a pair may pass qe)
        if (tid < kFxTile / 2 && q0 + 2 * tid < qe)
            __builtin_amdgcn_global_load_lds(
                (const void *)(reinterpret_cast<const uint4 *>(bm + q0) + tid),
                (__attribute__((address_space(3))) void *)(bdst), 16, 0, 0);
    };
    if (qb < qe) stage(t0, b0, qb);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    int buf = 0;
    for (int64_t q0 = qb; q0 < qe; q0 += kFxTile) {
        const bool more = q0 + kFxTile < qe;
        if (more) {
            if (buf)
                stage(t0, b0, q0 + kFxTile);
            else
                stage(t1, b1, q0 + kFxTile);
        }
        __builtin_amdgcn_sched_barrier(0);  // issue the copy before the contraction
        const double *tl = reinterpret_cast<const double *>(buf ? t1 : t0);
        const double *bl = reinterpret_cast<const double *>(buf ? b1 : b0);
        // A operand: t of grid point 16 wave + col ... rows of this wave
        const double *trow = tl + (16 * wave + col) * NP;
        v4d acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double t = trow[4 * s + grp];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(t, yf[c][s], acc[c], 0, 0, 0);
        }
        // FP64 output layout: lane l, register j holds row grp + 4 j of the
        // wave's 16 grid points, universe column col of block c (increasing q
        // in j, so a strict "<" keeps the lowest q among equal values)
        const int32_t qrow = (int32_t)q0 + 16 * wave + grp;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t q = qrow + 4 * j;
            if (q < qe) {
                const double bqv = bl[16 * wave + grp + 4 * j];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double v = (av[c] + bqv) - 2.0 * acc[c][j];
                    if (q == pv[c]) {  // kept in registers, stored once after the loop
                        cpv[c] = v;
                        hasp[c] = true;
                    }
                    if (v < best[c]) {
                        best[c] = v;
                        bq[c] = q;
                    }
                }
            }
        }
        if (more) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (hasp[c]) cp[td.r0 + 16 * c + col] = cpv[c];
    // minimum over the 4 lane groups (rows) of each wave, then over waves;
    // ties go to the lower q
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int sh = 16; sh <= 32; sh <<= 1) {
            const double ov = __shfl_xor(best[c], sh);
            const int32_t oq = __shfl_xor(bq[c], sh);
            if (ov < best[c] || (ov == best[c] && oq < bq[c])) {
                best[c] = ov;
                bq[c] = oq;
            }
        }
        if (grp == 0) {
            red_v[wave][16 * c + col] = best[c];
            red_q[wave][16 * c + col] = bq[c];
        }
    }
    __syncthreads();
    if (tid < kFxTile && tid < td.n) {
        double v = red_v[0][tid];
        int32_t q = red_q[0][tid];
        for (int w = 1; w < 4; ++w) {
            const double ov = red_v[w][tid];
            const int32_t oq = red_q[w][tid];
            if (ov < v || (ov == v && oq < q)) {
                v = ov;
                q = oq;
            }
        }
        const int64_t r = td.r0 + tid;
        cand_v[r * n_chunks + chunk] = v;
        cand_q[r * n_chunks + chunk] = q;
    }
}

// Merge the chunks of row r and write the universe's outputs (original order).
__global__ __launch_bounds__(256) void k_fixed_finish(
    int64_t R, int n_chunks, const double *__restrict__ cand_v,
    const int64_t *__restrict__ cand_q, const double *__restrict__ cp,
    const int64_t *__restrict__ order, const int64_t *__restrict__ p_of_row,
    double *__restrict__ dchi2, double *__restrict__ chi2_min, int64_t *__restrict__ argmin,
    double *__restrict__ chi2_p)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double v = __builtin_inf();
    int64_t q = INT64_MAX;
    for (int c = 0; c < n_chunks; ++c) {
        const double ov = cand_v[r * n_chunks + c];
        const int64_t oq = cand_q[r * n_chunks + c];
        if (ov < v || (ov == v && oq < q)) {
            v = ov;
            q = oq;
        }
    }
    const int64_t k = order[r];
    if (!(v < __builtin_inf())) q = p_of_row[r];  // no chi2 below +inf: Algorithm 1 keeps p
    dchi2[k] = cp[r] - v;
    chi2_min[k] = v;
    argmin[k] = q;
    chi2_p[k] = cp[r];
}

namespace {

struct Buf {
    void *p = nullptr;
    size_t n = 0;
    ~Buf()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t need(size_t bytes)
    {
        if (bytes <= n) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) n = bytes;
        return e;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

template <int NS>
hipError_t launch_fixed_min_ns(const FxTileDesc *tiles, int64_t n_tiles, const double *Y,
                               const double *a, const int64_t *p_of_row, const double *T,
                               const double *b, int64_t b_stride, int64_t G, int64_t q_per_chunk,
                               int n_chunks, double *cand_v, int64_t *cand_q, double *cp,
                               hipStream_t st)
{
    hipLaunchKernelGGL((k_fixed_min<NS>), dim3((unsigned)(n_tiles * n_chunks)), dim3(kFxThreads),
                       0, st, tiles, n_tiles, Y, a, p_of_row, T, b, b_stride, G, q_per_chunk,
                       n_chunks, cand_v, cand_q, cp);
    return hipGetLastError();
}

hipError_t launch_fixed_min(int ns, const FxTileDesc *tiles, int64_t n_tiles, const double *Y,
                            const double *a, const int64_t *p_of_row, const double *T,
                            const double *b, int64_t b_stride, int64_t G, int64_t q_per_chunk,
                            int n_chunks, double *cand_v, int64_t *cand_q, double *cp,
                            hipStream_t st)
{
    switch (ns) {
#define FC_CASE(n)                                                                                \
    case n:                                                                                       \
        return launch_fixed_min_ns<n>(tiles, n_tiles, Y, a, p_of_row, T, b, b_stride, G,          \
                                      q_per_chunk, n_chunks, cand_v, cand_q, cp, st);
        FC_CASE(1) FC_CASE(2) FC_CASE(3) FC_CASE(4) FC_CASE(5) FC_CASE(6) FC_CASE(7) FC_CASE(8)
        FC_CASE(9) FC_CASE(10) FC_CASE(11) FC_CASE(12) FC_CASE(13) FC_CASE(14) FC_CASE(15)
        FC_CASE(16)
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

template <int NS>
hipError_t launch_fixed_t_ns(const fc_grid *g, const int64_t *m_of_slot, int64_t n_slots,
                             int64_t b_stride, double *T, double *b, hipStream_t st)
{
    const int64_t n_qtiles = (g->G + 63) / 64;
    hipLaunchKernelGGL((k_fixed_t<NS>), dim3((unsigned)(n_slots * n_qtiles)), dim3(256), 0, st,
                       g->W64, g->S64, g->off, m_of_slot, g->N, g->G, n_qtiles, b_stride, T, b);
    return hipGetLastError();
}

hipError_t launch_fixed_t(int ns, const fc_grid *g, const int64_t *m_of_slot, int64_t n_slots,
                          int64_t b_stride, double *T, double *b, hipStream_t st)
{
    switch (ns) {
#define FC_CASE(n) \
    case n: return launch_fixed_t_ns<n>(g, m_of_slot, n_slots, b_stride, T, b, st);
        FC_CASE(1) FC_CASE(2) FC_CASE(3) FC_CASE(4) FC_CASE(5) FC_CASE(6) FC_CASE(7) FC_CASE(8)
        FC_CASE(9) FC_CASE(10) FC_CASE(11) FC_CASE(12) FC_CASE(13) FC_CASE(14) FC_CASE(15)
        FC_CASE(16)
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// One round over the rows listed in order[0..R) (universe k = order[r], all
// rows of a group contiguous and sharing matrix index m).  host_m[r] is the
// matrix grid index of row r, host_p[r] its true point.
static hipError_t fixed_round(const fc_grid *g, int64_t R, const std::vector<int64_t> &h_order,
                              const std::vector<int64_t> &h_m, const std::vector<int64_t> &h_p,
                              const double *d, double *dchi2, double *chi2_min, int64_t *argmin,
                              double *chi2_p, Buf *bufs, hipStream_t st)
{
    const int N = g->N, ns = (N + 3) / 4, np = 4 * ns;
    const int64_t G = g->G;
    // groups: runs of equal m; matrix slots batched so that t fits a budget
    const int64_t b_stride = G + (G & 1) + 2;  // even (16-byte rows) plus a pair of slack
    const size_t t_bytes_per_slot = sizeof(double) * ((size_t)G * np + b_stride);
    const size_t budget = size_t(4) << 30;
    const int64_t slots_max = std::max<int64_t>(1, (int64_t)(budget / t_bytes_per_slot));
    Buf &dOrder = bufs[0], &dM = bufs[1], &dP = bufs[2], &dY = bufs[3], &dA = bufs[4],
        &dT = bufs[5], &dB = bufs[6], &dSlotM = bufs[7], &dTiles = bufs[8], &dCv = bufs[9],
        &dCq = bufs[10], &dCp = bufs[11];
    hipError_t e;
    int64_t r_begin = 0;
    while (r_begin < R) {
        // rows r_begin .. r_end cover at most slots_max distinct m
        std::vector<int64_t> slot_m;
        std::vector<FxTileDesc> tiles;
        int64_t r = r_begin;
        while (r < R && (int64_t)slot_m.size() < slots_max) {
            const int64_t m = h_m[r];
            int64_t r2 = r;
            while (r2 < R && h_m[r2] == m) ++r2;
            const int32_t slot = (int32_t)slot_m.size();
            slot_m.push_back(m);
            for (int64_t t0 = r; t0 < r2; t0 += kFxTile) {
                FxTileDesc td;
                td.r0 = t0 - r_begin;
                td.n = (int32_t)std::min<int64_t>(kFxTile, r2 - t0);
                td.slot = slot;
                tiles.push_back(td);
            }
            r = r2;
        }
        const int64_t r_end = r, nr = r_end - r_begin, n_slots = (int64_t)slot_m.size();
        const int64_t n_tiles = (int64_t)tiles.size();
        // grid chunks: enough blocks to fill the chip, chunks of whole tiles
        static const int slots_res =  // queried once (thread-safe)
            resident_slots(reinterpret_cast<const void *>(&k_fixed_min<15>), kFxThreads);
        int n_chunks = (int)std::max<int64_t>(1, (4 * (int64_t)slots_res + n_tiles - 1) / n_tiles);
        const int64_t max_chunks = std::max<int64_t>(1, (G + kFxTile - 1) / kFxTile);
        n_chunks = (int)std::min<int64_t>(n_chunks, max_chunks);
        int64_t qpc = (G + n_chunks - 1) / n_chunks;
        qpc = ((qpc + kFxTile - 1) / kFxTile) * kFxTile;
        n_chunks = (int)((G + qpc - 1) / qpc);

        if ((e = dOrder.need(sizeof(int64_t) * nr)) != hipSuccess ||
            (e = dM.need(sizeof(int64_t) * nr)) != hipSuccess ||
            (e = dP.need(sizeof(int64_t) * nr)) != hipSuccess ||
            (e = dY.need(sizeof(double) * nr * np)) != hipSuccess ||
            (e = dA.need(sizeof(double) * nr)) != hipSuccess ||
            (e = dT.need(sizeof(double) * (size_t)n_slots * G * np)) != hipSuccess ||
            (e = dB.need(sizeof(double) * (size_t)n_slots * b_stride)) != hipSuccess ||
            (e = dSlotM.need(sizeof(int64_t) * n_slots)) != hipSuccess ||
            (e = dTiles.need(sizeof(FxTileDesc) * n_tiles)) != hipSuccess ||
            (e = dCv.need(sizeof(double) * nr * n_chunks)) != hipSuccess ||
            (e = dCq.need(sizeof(int64_t) * nr * n_chunks)) != hipSuccess ||
            (e = dCp.need(sizeof(double) * nr)) != hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(dOrder.p, h_order.data() + r_begin, sizeof(int64_t) * nr,
                                hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(dM.p, h_m.data() + r_begin, sizeof(int64_t) * nr,
                                hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(dP.p, h_p.data() + r_begin, sizeof(int64_t) * nr,
                                hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(dSlotM.p, slot_m.data(), sizeof(int64_t) * n_slots,
                                hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(dTiles.p, tiles.data(), sizeof(FxTileDesc) * n_tiles,
                                hipMemcpyHostToDevice, st)) != hipSuccess)
            return e;
        // chi2 at the true point is always met (p is a grid point); NaN until then
        hipLaunchKernelGGL(k_fixed_y, dim3((unsigned)((nr + 3) / 4)), dim3(256), 0, st, g->W64, d,
                           g->off, dOrder.as<int64_t>(), dM.as<int64_t>(), N, np, nr,
                           dY.as<double>(), dA.as<double>());
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_fixed_t(ns, g, dSlotM.as<int64_t>(), n_slots, b_stride, dT.as<double>(),
                                dB.as<double>(), st)) != hipSuccess)
            return e;
        if ((e = launch_fixed_min(ns, dTiles.as<FxTileDesc>(), n_tiles, dY.as<double>(),
                                  dA.as<double>(), dP.as<int64_t>(), dT.as<double>(),
                                  dB.as<double>(), b_stride, G, qpc, n_chunks, dCv.as<double>(),
                                  dCq.as<int64_t>(), dCp.as<double>(), st)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_fixed_finish, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st,
                           nr, n_chunks, dCv.as<double>(), dCq.as<int64_t>(), dCp.as<double>(),
                           dOrder.as<int64_t>(), dP.as<int64_t>(), dchi2, chi2_min, argmin,
                           chi2_p);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // the host vectors above are reused by the next batch
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        r_begin = r_end;
    }
    return hipSuccess;
}

hipError_t fixed_run(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                     int max_iter, double *dchi2, double *chi2_min, int64_t *argmin,
                     double *chi2_p, int64_t *m_final, int32_t *iters, hipStream_t st)
{
    const int64_t G = g->G;
    std::vector<int64_t> p(K), m(K), am(K);
    std::vector<int32_t> it(K, 0);
    hipError_t e;
    if ((e = hipMemcpyAsync(p.data(), p_idx, sizeof(int64_t) * K, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return e;
    for (int64_t k = 0; k < K; ++k) m[k] = p[k];
    std::vector<char> active(K, 1);
    Buf bufs[12];
    std::vector<int64_t> order, hm, hp, cnt;
    for (int round = 0;; ++round) {
        // counting sort of the active universes by m
        cnt.assign(G + 1, 0);
        int64_t R = 0;
        for (int64_t k = 0; k < K; ++k)
            if (active[k]) {
                ++cnt[m[k] + 1];
                ++R;
            }
        if (R == 0) break;
        for (int64_t q = 0; q < G; ++q) cnt[q + 1] += cnt[q];
        order.assign(R, 0);
        hm.assign(R, 0);
        hp.assign(R, 0);
        for (int64_t k = 0; k < K; ++k)
            if (active[k]) {
                const int64_t r = cnt[m[k]]++;
                order[r] = k;
                hm[r] = m[k];
                hp[r] = p[k];
            }
        if ((e = fixed_round(g, R, order, hm, hp, d, dchi2, chi2_min, argmin, chi2_p, bufs, st)) !=
            hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(am.data(), argmin, sizeof(int64_t) * K, hipMemcpyDeviceToHost,
                                st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return e;
        for (int64_t k = 0; k < K; ++k) {
            if (!active[k]) continue;
            if (round == max_iter || am[k] == m[k]) {
                active[k] = 0;
            } else {
                m[k] = am[k];
                it[k] = round + 1;
            }
        }
    }
    if (m_final &&
        (e = hipMemcpyAsync(m_final, m.data(), sizeof(int64_t) * K, hipMemcpyHostToDevice, st)) !=
            hipSuccess)
        return e;
    if (iters &&
        (e = hipMemcpyAsync(iters, it.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, st)) !=
            hipSuccess)
        return e;
    return hipStreamSynchronize(st);
}

}  // namespace fcx
