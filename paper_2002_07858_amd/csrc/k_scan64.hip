// k_scan64.hip -- the FP64 form of the scan on the FP64 matrix cores.
//
// chi2(d, q) = ||W_q (d - S_q)||^2 (Eq. (1) in factor form, Algorithm 2's
// arithmetic in FP64) for a tile of universes against a chunk of grid points,
// with Algorithm 1's strict-"<" running minimum in grid order.
//
// Contraction.  Per grid point the residual r = d - S_q is formed in FP64
// exactly as Algorithm 2 does (one rounding; r = 0 exactly when d = S_q), four
// bins at a time just before their tiles, and y = W_q r is computed on
// v_mfma_f64_4x4x4f64, whose four 4x4x4 blocks sit at lanes
// 16 k + 4 blk + {row | column}: A[i][k] at lane 16k + 4blk + i, B[k][j] at
// 16k + 4blk + j, D[i][j] at 16i + 4blk + j.  A is one 4 x 4 tile of W_q
// (the same in all four blocks), B holds four bins of 16 universes (four per
// block), D a 4-row block of y for them.  Only the nb (nb + 1) / 2 tiles on
// or below the diagonal are issued (120 at N = 57: 1920 MACs per evaluation
// for 1653 algorithmic).  A wave carries two sets of 16 universes, so every
// tile read from LDS feeds two MFMAs; a lane's accumulators hold one row of
// each 4-row block, chi2 is the lane's sum of squares plus a butterfly over
// the four row lanes (lanes l, l ^ 16, l ^ 32, l ^ 48), which adds the same
// operands in the same order in all of them.
//
// Records are double-buffered in LDS (direct global -> LDS loads issued one
// grid point ahead, one barrier per point).  The blocks of one universe tile
// split the grid into chunks; with several chunks each writes its (minimum,
// first q reaching it) to part[chunk][u], the chunk holding p writes
// chi2_p, and k_fp64_merge takes the minimum over the chunks in grid order
// with the same strict "<" -- the sequential scan's result exactly.
#include <utility>

#include "fc_internal.h"

namespace fcx {

namespace {

constexpr int kF64Waves = 4;                       // waves per block
constexpr int kF64Sets = 2;                        // sets of 16 universes per wave
constexpr int kF64Univ = 16 * kF64Sets * kF64Waves;  // universes per block (128)
constexpr int64_t kF64ChunkMax = 2048;                // grid points per block at most
constexpr size_t kF64PartsMax = size_t(2) << 30;      // bytes of chunk partials at most

template <int N>
struct F64Acc {
    static constexpr int NB = f64_nb(N), NBE = f64_nbe(N), L = f64_lead(N);
    double d[kF64Sets][NB];    // universes: bin 4 kb + lane/16 - P of universe lane%16
    double dl[kF64Sets][L > 0 ? L : 1];  // the lead bins 0 .. L-1 of universe lane%16
    double sig[NBE];           // S_q at the lane's bins (one grid point)
    double r[kF64Sets][NB];    // residuals of the current bin block
    double acc[kF64Sets][NB];  // y rows 4 r + lane/16 of universe lane%16
};

// MFMA of tile t for both sets.  The first tile of a bin block forms its
// residuals; the first bin block starts the accumulators from zero, or from
// the lead columns' products when those are on the vector ALUs.
template <int N, int t>
__device__ __forceinline__ void f64_tile(F64Acc<N> &s, double a)
{
    constexpr int kb = f64_tile_kb(N, t), r = f64_tile_r(N, t);
    if constexpr (r == kb) {
#pragma unroll
        for (int c = 0; c < kF64Sets; ++c) s.r[c][kb] = s.d[c][kb] - s.sig[kb];
    }
#pragma unroll
    for (int c = 0; c < kF64Sets; ++c) {
        if constexpr (kb == 0)
            s.acc[c][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, s.r[c][kb], 0.0, 0, 0, 0);
        else
            s.acc[c][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, s.r[c][kb], s.acc[c][r], 0, 0, 0);
    }
}

template <int N, int... p>
__device__ __forceinline__ void f64_tiles(F64Acc<N> &s, const double2 *__restrict__ rec, int pos,
                                          std::integer_sequence<int, p...>)
{
    constexpr int nt = f64_ntile(N);
    (
        [&] {
            const double2 a = rec[p * 16 + pos];
            f64_tile<N, 2 * p>(s, a.x);
            if constexpr (2 * p + 1 < nt) f64_tile<N, 2 * p + 1>(s, a.y);
        }(),
        ...);
}

// Sum of x over the lanes l, l ^ 16, l ^ 32, l ^ 48 for two values a (set 0)
// and b (set 1): lanes < 32 get set 0's sum, lanes >= 32 set 1's.  The upper
// half of a is swapped with the lower half of b, then 16-lane rows pair up
// through a swizzle (lane l reads lane l ^ 16), which runs on the LDS unit
// and so takes no vector-ALU time from the FP64 MFMAs.
__device__ __forceinline__ double f64_row_sum(double a, double b)
{
    const uint2 ua = __builtin_bit_cast(uint2, a), ub = __builtin_bit_cast(uint2, b);
    const auto lo = __builtin_amdgcn_permlane32_swap(ua.x, ub.x, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(ua.y, ub.y, false, false);
    const double a2 = __builtin_bit_cast(double, make_uint2(lo[0], hi[0]));
    const double b2 = __builtin_bit_cast(double, make_uint2(lo[1], hi[1]));
    const double h = a2 + b2;  // lane l < 32: a_l + a_{l+32}; lane l >= 32: b_{l-32} + b_l
    const uint2 uh = __builtin_bit_cast(uint2, h);
    // bit-mode swizzle: and 0x1f, or 0, xor 0x10 within each 32-lane half
    const uint32_t sx = (uint32_t)__builtin_amdgcn_ds_swizzle((int)uh.x, 0x401F);
    const uint32_t sy = (uint32_t)__builtin_amdgcn_ds_swizzle((int)uh.y, 0x401F);
    return h + __builtin_bit_cast(double, make_uint2(sx, sy));
}

template <int N>
__global__ __launch_bounds__(64 * kF64Waves) __attribute__((amdgpu_waves_per_eu(3))) void
k_scan_f64m(const uint4 *__restrict__ R64, const double *__restrict__ d,
            const int64_t *__restrict__ p_idx, int64_t K, int64_t q0, int64_t nq,
            int64_t n_utiles, int64_t q_per_chunk, Fp64Part *__restrict__ part,
            double *__restrict__ dchi2, double *__restrict__ chi2_min,
            int64_t *__restrict__ argmin, double *__restrict__ chi2_p)
{
    constexpr int NB = f64_nb(N), P = f64_pad(N), NBE = f64_nbe(N), L = f64_lead(N);
    constexpr int REC = f64_rec_units(N);  // 16-byte units per record
    __shared__ uint4 lds[2][REC];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t utile = blockIdx.x % n_utiles, chunk = blockIdx.x / n_utiles;
    const int64_t qb = q0 + chunk * q_per_chunk;
    const int64_t qe = (qb + q_per_chunk < q0 + nq) ? qb + q_per_chunk : q0 + nq;
    const int64_t ubase = utile * kF64Univ + (int64_t)wave * 16 * kF64Sets;

    if (qb < qe) record_to_lds<REC, 64 * kF64Waves>(R64 + qb * (int64_t)REC, lds[0], tid);

    // stage d for both sets: bin 4 kb + lane/16 - P of universe lane%16, and
    // the lead bins of the same universe (loads from clamped, in-bounds
    // addresses; padding bins and idle lanes select 0)
    F64Acc<N> s;
#pragma unroll
    for (int c = 0; c < kF64Sets; ++c) {
        const int64_t u = ubase + 16 * c + (lane & 15);
        const bool act = u < K;
        const double *du = d + (act ? u : K - 1) * N;
#pragma unroll
        for (int kb = f64_k0(N); kb < NB; ++kb) {
            const int j = 4 * kb + (lane >> 4) - P;
            const double v = du[j < 0 ? 0 : j];
            s.d[c][kb] = (act && j >= 0) ? v : 0.0;
        }
#pragma unroll
        for (int b = 0; b < L; ++b) s.dl[c][b] = act ? du[b] : 0.0;
    }
    // the universe this lane tracks after the row butterfly
    const int64_t u_own = ubase + 16 * (lane >> 5) + (lane & 15);
    const bool own_act = u_own < K;
    const int64_t p = own_act ? p_idx[u_own] : -1;
    double best = __builtin_inf();
    int64_t qbest = p;
    double cp = __builtin_nan("");
    const int pos = 4 * (lane >> 4) + (lane & 3);

    int buf = 0;
    for (int64_t q = qb; q < qe; ++q) {
        wait_record_loads();
        __syncthreads();  // record q is in lds[buf]; every wave is done with lds[buf ^ 1]
        if (q + 1 < qe)
            record_to_lds<REC, 64 * kF64Waves>(R64 + (q + 1) * (int64_t)REC, lds[buf ^ 1], tid);
        const double *rec = reinterpret_cast<const double *>(lds[buf]);
        {
            // this lane's signal bins (g = lane / 16)
            const double2 *sg =
                reinterpret_cast<const double2 *>(rec + f64_sig_double(N) + (lane >> 4) * NBE);
#pragma unroll
            for (int k = 0; k < NBE / 2; ++k) {
                const double2 v = sg[k];
                s.sig[2 * k] = v.x;
                s.sig[2 * k + 1] = v.y;
            }
        }
        if constexpr (L > 0) {
            // lead columns on the vector ALUs: every accumulator starts at
            // sum_b W'[row][P + b] (d_b - S_q[b]) for the lane's own universe
            double rl[kF64Sets][L];
#pragma unroll
            for (int b = 0; b < L; ++b) {
                const double sb = rec[f64_sig_double(N) + (P + b) * NBE];  // S_q[b]: kb 0, g = P + b
#pragma unroll
                for (int c = 0; c < kF64Sets; ++c) rl[c][b] = s.dl[c][b] - sb;
            }
#pragma unroll
            for (int b = 0; b < L; ++b) {
                const double2 *wl = reinterpret_cast<const double2 *>(
                    rec + f64_lead_double(N) + (b * 4 + (lane >> 4)) * NBE);
#pragma unroll
                for (int k = 0; k < NBE / 2; ++k) {
                    const double2 w = wl[k];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int r = 2 * k + h;
                        if (r < NB) {
                            const double wv = h ? w.y : w.x;
#pragma unroll
                            for (int c = 0; c < kF64Sets; ++c)
                                s.acc[c][r] = b ? fma(wv, rl[c][b], s.acc[c][r]) : wv * rl[c][b];
                        }
                    }
                }
            }
        }
        f64_tiles<N>(s, reinterpret_cast<const double2 *>(rec), pos,
                     std::make_integer_sequence<int, f64_npair(N)>{});
        double sq[kF64Sets];
#pragma unroll
        for (int c = 0; c < kF64Sets; ++c) {
            double a = s.acc[c][0] * s.acc[c][0];
#pragma unroll
            for (int r = 1; r < NB; ++r) a = fma(s.acc[c][r], s.acc[c][r], a);
            sq[c] = a;
        }
        const double chi2 = f64_row_sum(sq[0], sq[1]);
        if (q == p) cp = chi2;
        if (chi2 < best) {
            best = chi2;
            qbest = q;
        }
        buf ^= 1;
    }
    if (!own_act || (lane & 16)) return;  // one lane per universe writes
    if (part) {
        part[chunk * K + u_own] = Fp64Part{best, qbest};
        if (p >= qb && p < qe) chi2_p[u_own] = cp;
        return;
    }
    if (chi2_min) chi2_min[u_own] = best;
    if (argmin) argmin[u_own] = qbest;
    if (chi2_p) chi2_p[u_own] = cp;
    dchi2[u_own] = cp - best;
}

}  // namespace

// Merge of the FP64 chunks: one wave per universe.  Lane l takes chunks l,
// l + 64, ... in grid order with the strict "<", then the wave reduces the 64
// (value, q) pairs by shuffles, keeping the lower q among equal values: the
// chunks partition the grid in order, so that is the earlier chunk, and the
// result is the sequential scan's.  Chunk values are never NaN (a NaN chi2
// never passes "<"), and a chunk with no finite value reports (+inf, p).  A
// true point outside [0, G) was owned by no chunk: chi2_p = NaN.  chi2_min
// and argmin may be nullptr; chi2_p holds the owners' values on entry.
__global__ __launch_bounds__(256) void k_fp64_merge(const Fp64Part *__restrict__ part,
                                                   int64_t n_chunks, const int64_t *__restrict__ p_idx,
                                                   int64_t K, int64_t G, double *__restrict__ dchi2,
                                                   double *__restrict__ chi2_min,
                                                   int64_t *__restrict__ argmin,
                                                   double *__restrict__ chi2_p)
{
    const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (u >= K) return;  // uniform per wave
    const int64_t p = p_idx[u];
    double best = __builtin_inf();
    int64_t qbest = p;
    for (int64_t c = lane; c < n_chunks; c += 64) {
        const Fp64Part x = part[c * K + u];
        if (x.v < best) {
            best = x.v;
            qbest = x.q;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(best, off, 64);
        const int64_t oq = __shfl_xor(qbest, off, 64);
        if (ov < best || (ov == best && oq < qbest)) {
            best = ov;
            qbest = oq;
        }
    }
    if (lane != 0) return;
    const double cp = (p >= 0 && p < G) ? chi2_p[u] : __builtin_nan("");
    if (chi2_min) chi2_min[u] = best;
    if (argmin) argmin[u] = qbest;
    chi2_p[u] = cp;
    dchi2[u] = cp - best;
}

// Initial chi2_p of a chunked scan: NaN for universes whose true point no
// chunk owns.
__global__ __launch_bounds__(256) void k_fill_nan(int64_t K, double *__restrict__ x)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < K) x[u] = __builtin_nan("");
}

namespace {

template <int N>
hipError_t launch_f64m_n(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                          Fp64Part *scratch, size_t scratch_bytes, double *dchi2,
                          double *chi2_min, int64_t *argmin, double *chi2_p, hipStream_t st)
{
    static const int slots =
        resident_slots(reinterpret_cast<const void *>(&k_scan_f64m<N>), 64 * kF64Waves);
    const int64_t G = g->G;
    // chunks: the fewest that fill the resident slots with a small tail
    ScanGeometry sg = scan_geometry(K, G, slots, kF64Univ);
    int64_t chunks = sg.n_qchunks, qpc = sg.q_per_chunk;
    // then shorter chunks, of at most kF64ChunkMax points, as far as the
    // dispatch size and the partials' bound allow (c5: 9.11 s against 9.27 s
    // with the 11 chunks of 95 326 points above; same results bit for bit)
    if (qpc > kF64ChunkMax) {
        const int64_t by_dispatch = (int64_t(1) << 23) / (sg.n_utiles > 0 ? sg.n_utiles : 1);
        const int64_t by_parts = (int64_t)(kF64PartsMax / (sizeof(Fp64Part) * (size_t)K));
        int64_t nc = (G + kF64ChunkMax - 1) / kF64ChunkMax;
        if (nc > by_dispatch) nc = by_dispatch;
        if (nc > by_parts) nc = by_parts;
        if (nc > chunks) {
            qpc = (G + nc - 1) / nc;
            chunks = (G + qpc - 1) / qpc;
        }
    }
    // the partials must fit the scratch (library-owned or the caller's)
    const int64_t max_chunks = (int64_t)(scratch_bytes / (sizeof(Fp64Part) * (size_t)K));
    Fp64Part *part = nullptr;
    bool own = false;
    if (chunks > 1) {
        if (scratch) {
            if (chunks > max_chunks) {
                chunks = max_chunks < 1 ? 1 : max_chunks;
                qpc = (G + chunks - 1) / chunks;
                chunks = (G + qpc - 1) / qpc;
            }
            if (chunks > 1) part = scratch;
        } else {
            hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&part),
                                          sizeof(Fp64Part) * (size_t)chunks * (size_t)K, st);
            if (e != hipSuccess) return e;
            own = true;
        }
    }
    if (chunks <= 1) {
        chunks = 1;
        qpc = G;
    }
    const int64_t blocks = sg.n_utiles * chunks;
    if (part)
        hipLaunchKernelGGL(k_fill_nan, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, K,
                           chi2_p);
    {
        ProfScope prof(st, "k_scan_f64m");
        hipLaunchKernelGGL(k_scan_f64m<N>, dim3((unsigned)blocks), dim3(64 * kF64Waves), 0, st,
                           g->R64, d, p_idx, K, (int64_t)0, G, sg.n_utiles, qpc, part, dchi2,
                           chi2_min, argmin, chi2_p);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && part) {
        hipLaunchKernelGGL(k_fp64_merge, dim3((unsigned)((K + 3) / 4)), dim3(256), 0, st, part,
                           chunks, p_idx, K, G, dchi2, chi2_min, argmin, chi2_p);
        e = hipGetLastError();
    }
    if (own) {
        const hipError_t ef = hipFreeAsync(part, st);
        if (e == hipSuccess) e = ef;
    }
    return e;
}

}  // namespace

hipError_t launch_scan_fp64(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                            double *dchi2, double *chi2_min, int64_t *argmin, double *chi2_p,
                            hipStream_t st, Fp64Part *scratch, size_t scratch_bytes)
{
    if (K <= 0) return hipSuccess;
    switch (g->N) {
#define FC_CASE(n)                                                                                \
    case n:                                                                                       \
        return launch_f64m_n<n>(g, K, d, p_idx, scratch, scratch_bytes, dchi2, chi2_min, argmin,  \
                                chi2_p, st);
#define FC_CASE8(b) FC_CASE(b + 1) FC_CASE(b + 2) FC_CASE(b + 3) FC_CASE(b + 4) \
                    FC_CASE(b + 5) FC_CASE(b + 6) FC_CASE(b + 7) FC_CASE(b + 8)
        FC_CASE8(0) FC_CASE8(8) FC_CASE8(16) FC_CASE8(24) FC_CASE8(32) FC_CASE8(40) FC_CASE8(48)
        FC_CASE8(56)
#undef FC_CASE8
#undef FC_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fcx
