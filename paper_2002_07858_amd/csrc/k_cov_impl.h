// k_cov_impl.h -- per-grid-point covariance, FP64 Cholesky and inverse factor
// (the kernel template; instantiated per padded bin count NP in the
// k_cov_np_*.hip files, launched from k_cov.hip).
//
// For grid point q (Section 1: M in Eq. (1) is the inverse of a covariance
// carrying statistical and systematic uncertainties):
//     Sigma_q = diag(stat_q) + F o (S_q S_q^T)
//     L_q L_q^T = Sigma_q          right-looking Cholesky, FP64
//     W_q = L_q^{-1}               forward substitution, FP64
// so that Sigma_q^{-1} = W_q^T W_q and chi2 = ||W_q r||^2.  This is the step
// whose conditioning needs FP64; the scan forms only ever see W_q.
//
// One wave per grid point, the matrix in registers: bins are padded to NP, a
// multiple of four (padding rows and columns of Sigma_q are those of the
// identity), and the kernel is instantiated per NP with every loop over rows
// and columns unrolled, so that lane i keeps a whole row (then a whole column)
// in NP register pairs.
//   * Cholesky, lane i = row i of the trailing matrix: at step j every lane
//     writes its element of column j to LDS and reads the column back as
//     broadcasts (16-byte reads); the pivot p = A[j][j] gives
//     L[.][j] = A[.][j] / sqrt(p), and the trailing update
//     A[i][k] -= (A[i][j] / p) A[k][j] is one FMA per register.  The columns
//     stay in LDS (even lengths, 16-byte aligned).
//   * Inversion, lane i = column i of W (L w = e_i): forward substitution in
//     axpy form over the same stored columns, w_j = s_j / L[j][j], then
//     s_r -= L[r][j] w_j for r > j, one FMA per register.
// Every column read is a wave-wide broadcast used by one FMA per lane: the LDS
// reads (NP^2 / 2 doubles per point and pass) and the FP64 FMAs are of the same
// order, and with about two waves per SIMD the per-step chain (store,
// broadcast, pivot) is what the waves mostly wait on.  W_q
// then goes to HBM straight from the registers (packed rows: lanes write
// consecutive addresses) and, as packed rows, into LDS, from where each
// requested record form is written as gathers through a per-N map
// (fc_internal.h), one coalesced store per element.
#pragma once
#include <stdint.h>

#include <type_traits>

#include "fc_internal.h"

namespace fcx {

// Column j of the factorisation in LDS: rows j .. NP-1, padded to an even count.
__host__ __device__ constexpr int cov_col_len(int NP, int j) { return (NP - j + 1) & ~1; }
__host__ __device__ constexpr int cov_col_off(int NP, int j)
{
    int o = 0;
    for (int jj = 0; jj < j; ++jj) o += cov_col_len(NP, jj);
    return o;
}
// LDS doubles of one point: the column store (later W_q's packed rows), then
// S_q, S_q - fl32(S_q), S_q - o and 1/L[j][j], 64 each.
__host__ __device__ constexpr int cov_region(int NP)
{
    return cov_col_off(NP, NP) > NP * (NP + 1) / 2 ? cov_col_off(NP, NP)
                                                    : ((NP * (NP + 1) / 2 + 1) & ~1);
}
__host__ __device__ constexpr int cov_lds_doubles(int NP) { return cov_region(NP) + 4 * 64; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// hi + lo split of eight FP32 values into two 16-byte fragments (round to
// nearest even for both halves).
template <bool FP16>
__device__ inline void split8(const float (&x)[8], uint4 &hi, uint4 &lo)
{
    if constexpr (FP16) {
        f16x8 h, l;
        for (int e = 0; e < 8; ++e) {
            h[e] = (_Float16)x[e];
            l[e] = (_Float16)(x[e] - (float)h[e]);
        }
        hi = __builtin_bit_cast(uint4, h);
        lo = __builtin_bit_cast(uint4, l);
    } else {
        bf16x8 h, l;
        for (int e = 0; e < 8; ++e) {
            h[e] = (__bf16)x[e];
            l[e] = (__bf16)(x[e] - (float)h[e]);
        }
        hi = __builtin_bit_cast(uint4, h);
        lo = __builtin_bit_cast(uint4, l);
    }
}

// Materialise x here: without it the compiler may defer a register's updates
// to its first use and keep every step's column values live until then.
__device__ __forceinline__ void pin(double &x) { asm volatile("" : "+v"(x)); }

// for (I = B; I < E; ++I) fn(integral_constant<I>), expanded at compile time
// (the loops over a register row must be unrolled for its indices to be
// static; the unroller gives up on the larger bin counts).
template <int B, int E, class Fn>
__device__ __forceinline__ void static_for(Fn &&fn)
{
    if constexpr (B < E) {
        fn(std::integral_constant<int, B>{});
        static_for<B + 1, E>(fn);
    }
}

// One step of either pass: a[k] = fma(-mul, c[k], a[k]) for J < k < NP, with
// c = column J of the factorisation, read from `col` as 16-byte broadcasts in
// chunks of kCovChunk pairs, two chunks in flight ahead of the FMAs; mul comes
// from mulfn(first pair) (the pivot's pair).
constexpr int kCovChunk = 3;

template <int NP, int J, class MulFn>
__device__ __forceinline__ void cov_update(const double2 *col, double (&a)[NP], MulFn mulfn)
{
    constexpr int np = cov_col_len(NP, J) / 2;
    constexpr int nch = (np + kCovChunk - 1) / kCovChunk;
    double2 buf[2][kCovChunk];
    static_for<0, 2 * kCovChunk>([&](auto hm) {
        constexpr int x = decltype(hm)::value;
        if constexpr (x < np) buf[x / kCovChunk][x % kCovChunk] = col[x];
    });
    const double mul = mulfn(buf[0][0]);
    static_for<0, nch>([&](auto chc) {
        constexpr int ch = decltype(chc)::value;
        __builtin_amdgcn_sched_barrier(0);
        static_for<0, kCovChunk>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            constexpr int k = J + 2 * (ch * kCovChunk + m);
            if constexpr (ch * kCovChunk + m < np) {
                if constexpr (k > J && k < NP) {
                    a[k] = fma(-mul, buf[ch & 1][m].x, a[k]);
                    pin(a[k]);
                }
                if constexpr (k + 1 < NP) {
                    a[k + 1] = fma(-mul, buf[ch & 1][m].y, a[k + 1]);
                    pin(a[k + 1]);
                }
            }
        });
        __builtin_amdgcn_sched_barrier(0);
        static_for<0, kCovChunk>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            if constexpr ((ch + 2) * kCovChunk + m < np)
                buf[ch & 1][m] = col[(ch + 2) * kCovChunk + m];
        });
    });
}

// One record element through its map entry.
__device__ __forceinline__ double cov_gather(int m, const double *Wl, const double *Sl)
{
    return (m < 0) ? 0.0 : (m >= kMapSig ? Sl[m - kMapSig] : Wl[m]);
}

// One split-form record (see fc_internal.h) from W_q's packed rows in LDS;
// wmax = max |W_q| (FP16 range).  Each fragment element is one gathered W_q
// entry, scaled, rounded to the 16-bit type (hi) or, marked kMapLo, the rest
// of that rounding (lo).
template <bool FP16>
__device__ void write_split_record(const double *Wl, const double *sdo, const int16_t *map, int N,
                                   int ed, double wmax, uint4 *rq, int i)
{
    const int code = split_code(N);
    const int eq = (FP16 && wmax > 0.0) ? 13 - ilogb(wmax) : 0;
    const int nf = code_nfrag(code);
    for (int u = i; u < nf * 64; u += 64) {
        const int16_t *mu = map + 8 * u;
        float x[8];
        bool lo[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int m = mu[e];
            lo[e] = m >= 0 && (m & kMapLo) != 0;
            x[e] = (m < 0) ? 0.0f : (float)ldexp(Wl[m & (kMapLo - 1)], eq);
        }
        uint4 hi, lw;
        split8<FP16>(x, hi, lw);
        const uint32_t *ph = reinterpret_cast<const uint32_t *>(&hi);
        const uint32_t *pl = reinterpret_cast<const uint32_t *>(&lw);
        uint32_t w[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint32_t m0 = lo[2 * h] ? 0x0000ffffu : 0u;
            const uint32_t m1 = lo[2 * h + 1] ? 0xffff0000u : 0u;
            w[h] = (ph[h] & ~(m0 | m1)) | (pl[h] & (m0 | m1));
        }
        rq[u] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    // u_q = W_q (S_q - o) in FP64, in the accumulator's row order [l/16][g][j]
    {
        const int gl = i >> 4, g = (i >> 2) & 3, j = i & 3;
        const int row = split_row0(N, g) + 4 * gl + j;
        double u = 0.0;
        if (g < split_nb(N) && row < split_row0(N, g + 1)) {
            const double *wr = Wl + row * (row + 1) / 2;
#pragma unroll 4
            for (int k = 0; k <= row; ++k) u += wr[k] * sdo[k];
        }
        reinterpret_cast<float *>(rq + code_u_unit(code))[i] = (float)ldexp(-u, eq + ed);
    }
    const int su = code_scale_unit(code), ru = code_rec_units(code);
    if (i == 0) rq[su] = make_uint4(__float_as_uint(ldexpf(1.0f, -2 * (eq + ed))), 0u, 0u, 0u);
    for (int u = su + 1 + i; u < ru; u += 64) rq[u] = make_uint4(0u, 0u, 0u, 0u);
}

template <int NP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_cov_build(
    const double *__restrict__ S64, const double *__restrict__ F, const double *__restrict__ stat,
    const double *__restrict__ off, int N_arg, int64_t G, int stat_mode, uint32_t forms, int ns,
    int ed16, const int16_t *__restrict__ maps, double *__restrict__ W64, uint4 *__restrict__ R64,
    uint4 *__restrict__ R32, uint4 *__restrict__ RB16, uint4 *__restrict__ RH16,
    unsigned long long *__restrict__ bad_q)
{
    static_assert(NP % 4 == 0 && NP >= 4 && NP <= 64, "NP: a multiple of four up to 64");
    extern __shared__ double2 smem2[];
    double *const Lc = reinterpret_cast<double *>(smem2);  // column store, then W_q's rows
    double *const Sl = Lc + cov_region(NP);                 // S_q
    double *const sdl = Sl + 64;                            // S_q - fl32(S_q)
    double *const sdo = sdl + 64;                           // S_q - o
    double *const rlv = sdo + 64;                           // 1 / L[j][j]
    const double stat_i =
        ((int)threadIdx.x < N_arg && stat_mode != FC_STAT_PEARSON) ? stat[threadIdx.x] : 0.0;
    const double off_i = ((int)threadIdx.x < N_arg) ? off[threadIdx.x] : 0.0;

    for (int64_t q = blockIdx.x; q < G; q += gridDim.x) {
        // the lane index and N re-read per point: everything derived from them
        // (NP addresses and predicates) would otherwise be hoisted out of the
        // loop and held in registers across it
        int i = threadIdx.x, N = N_arg;
        asm volatile("" : "+v"(i), "+s"(N));
        const int16_t *map64 = maps;
        const int16_t *map32 = map64 + 2 * f64_rec_units(N);
        const int16_t *map16 = map32 + 4 * rec_w_units(ns);
        const double *Sq = S64 + q * N;
        const double si = (i < N) ? Sq[i] : 0.0;
        Sl[i] = si;
        sdl[i] = si - (double)(float)si;
        sdo[i] = si - off_i;
        __builtin_amdgcn_wave_barrier();

        // ---- row i of Sigma_q (F is symmetric: lanes read a column of it) ----
        // (the column's base is re-derived per point, so that its NP addresses
        // are not kept live across the loop over points)
        const double *Fi = F + i;
        double a[NP];
        static_for<0, NP / 2>([&](auto kc) {
            constexpr int k = 2 * decltype(kc)::value;
            const double2 sk = smem2[cov_region(NP) / 2 + k / 2];
            a[k] = (i < N && k < N) ? Fi[k * N] * (si * sk.x) : 0.0;
            a[k + 1] = (i < N && k + 1 < N) ? Fi[(k + 1) * N] * (si * sk.y) : 0.0;
            if constexpr (k % 8 == 6) __builtin_amdgcn_sched_barrier(0);  // 8 loads in flight
        });
        const double dg = (i < N) ? ((stat_mode == FC_STAT_PEARSON) ? si : stat_i) : 1.0;
        static_for<0, NP>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            a[k] = (k == i) ? a[k] + dg : a[k];
        });

        // ---- right-looking Cholesky, lane i = row i --------------------------
        int bad = 0;  // a pivot <= 0 or NaN (uniform)
        static_for<0, NP>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            double *col = Lc + cov_col_off(NP, j);
            if (i >= j && i < j + cov_col_len(NP, j)) col[i - j] = a[j];
            __builtin_amdgcn_wave_barrier();
            cov_update<NP, j>(reinterpret_cast<const double2 *>(col), a, [&](double2 p0) {
                const double piv = p0.x;
                bad |= (piv > 0.0) ? 0 : 1;
                asm volatile("" : "+v"(bad));  // folded now, not as NP masks at the end
                const double pv = (piv > 0.0) ? piv : 1.0;
                // 1 / sqrt(pv): the hardware estimate and two Newton steps,
                // y <- y (3/2 - (pv/2) y^2) (a short chain; every step waits
                // on it), and 1 / pv as its square
                const double h = 0.5 * pv;
                double y = __builtin_amdgcn_rsq(pv);
                y = y * fma(-h * y, y, 1.5);
                y = y * fma(-h * y, y, 1.5);
                if (i == 0) rlv[j] = y;
                return (i > j) ? a[j] * (y * y) : 0.0;
            });
        });
        if (bad) {  // uniform
            if (i == 0) atomicMin(bad_q, (unsigned long long)q);
            __builtin_amdgcn_wave_barrier();
            continue;
        }

        // ---- W = L^{-1}, lane i = column i: L w = e_i -------------------------
        // L[r][j] = c[r] rl with rl = 1 / L[j][j]: w_j = s_j rl, then
        // s_r -= c[r] (rl w_j) for r > j
        static_for<0, NP>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            a[r] = (r == i) ? 1.0 : 0.0;
        });
        __builtin_amdgcn_wave_barrier();
        static_for<0, NP>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const double rl = rlv[j];
            cov_update<NP, j>(reinterpret_cast<const double2 *>(Lc + cov_col_off(NP, j)), a,
                              [&](double2) {
                                  const double w = a[j] * rl;
                                  a[j] = w;
                                  return w * rl;
                              });
        });

        // ---- W_q: HBM (packed rows) and LDS (packed rows, over the columns) ----
        double wmax = 0.0;
        double *Wq = (forms & FC_FORM_FP64) ? W64 + q * ((int64_t)N * (N + 1) / 2) : nullptr;
        __builtin_amdgcn_wave_barrier();
        static_for<0, NP>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            if (r < N && i <= r) {
                const int at = r * (r + 1) / 2 + i;
                Lc[at] = a[r];
                if (Wq) Wq[at] = a[r];
                wmax = fmax(wmax, fabs(a[r]));
            }
            if constexpr (r % 8 == 7) __builtin_amdgcn_sched_barrier(0);
        });
        __builtin_amdgcn_wave_barrier();

        // ---- the requested record forms ----------------------------------------
        if (forms & FC_FORM_FP64) {
            double *rq = reinterpret_cast<double *>(R64 + q * (int64_t)f64_rec_units(N));
            const int n = 2 * f64_rec_units(N);
            for (int e = i; e < n; e += 64) rq[e] = cov_gather(map64[e], Lc, Sl);
        }
        if (forms & FC_FORM_FP32) {
            uint4 *rq = R32 + q * (int64_t)rec_units(ns);
            float *Wf = reinterpret_cast<float *>(rq);
            const int n = 4 * rec_w_units(ns);
            for (int e = i; e < n; e += 64) Wf[e] = (float)cov_gather(map32[e], Lc, Sl);
            // FP32 part of the signal (real bin order), then minus W_q times
            // its rounding error (padded row order)
            float *Sp = reinterpret_cast<float *>(rq + rec_w_units(ns));
            Sp[i] = (i < N) ? (float)si : 0.0f;
            const int rr = i - fp32_pad(ns, N);
            double cv = 0.0;
            if (rr >= 0 && rr < N) {
                const double *wr = Lc + rr * (rr + 1) / 2;
#pragma unroll 4
                for (int kk = 0; kk <= rr; ++kk) cv -= wr[kk] * sdl[kk];
            }
            Sp[64 + i] = (float)cv;
        }
        if (forms & (FC_FORM_SPLIT_BF16 | FC_FORM_SPLIT_FP16)) {
            for (int m = 32; m > 0; m >>= 1) wmax = fmax(wmax, __shfl_xor(wmax, m));
            const int64_t sru = split_rec_units(N);
            if (forms & FC_FORM_SPLIT_BF16)
                write_split_record<false>(Lc, sdo, map16, N, 0, wmax, RB16 + q * sru, i);
            if (forms & FC_FORM_SPLIT_FP16)
                write_split_record<true>(Lc, sdo, map16, N, ed16, wmax, RH16 + q * sru, i);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <int NP>
hipError_t launch_cov_np(const fc_grid *g, const double *F, const double *stat,
                                int stat_mode, uint32_t forms, const int16_t *maps, double *W64,
                                uint4 *R64, uint4 *R32, uint4 *RB16, uint4 *RH16,
                                unsigned long long *bad_q, hipStream_t st)
{
    const int64_t blocks = g->G < 65536 ? g->G : 65536;
    ProfScope prof(st, "k_cov_build");
    hipLaunchKernelGGL(k_cov_build<NP>, dim3((unsigned)blocks), dim3(64),
                       sizeof(double) * cov_lds_doubles(NP), st, g->S64, F, stat, g->off, g->N,
                       g->G, stat_mode, forms, g->ns, g->ed16, maps, W64, R64, R32, RB16, RH16,
                       bad_q);
    return hipGetLastError();
}

}  // namespace fcx
