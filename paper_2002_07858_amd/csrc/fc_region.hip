// fc_region.hip -- the Feldman-Cousins confidence region with per-point
// universe counts.
//
// Section 2 builds the Delta chi^2 distribution of every grid point p from
// N_univ universes drawn at p; the paper's closing section proposes letting
// N_univ differ between points so that large counts are spent only near the
// eventual contour.  This driver does that in rounds, entirely with the
// library's device paths (universe generation, scan, order statistics):
//
//   round 0   every point gets K0 universes (indices 0 .. K0-1 of its stream);
//   each round  scan the new universes, take the critical values
//             x_(ceil(alpha K)) over all K(p) universes of each point, and the
//             band [x_(j - delta), x_(j + delta)] around them,
//             j = ceil(alpha K), delta = ceil(z sqrt(K alpha (1 - alpha)))
//             (a z-sigma interval for the rank of the alpha-quantile);
//   a point is undecided while Delta chi^2 of the data at p lies inside the
//             band for some alpha; undecided points below K_max double K(p)
//             with universes K(p) .. 2K(p)-1 and go round again.
//
// Every point's Delta chi^2 values live in one device array (K_max slots per
// point); a round's new universes are drawn, scanned and scattered in batches.
// The result: the critical values, the acceptance dchi2_data(p) <= crit, and
// the universe count each point ended with.
#include "fc_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace fcx {

// store[slot[k] * K_max + u_first[k] + (r - seg_off[k])] = dchi2[r]
__global__ __launch_bounds__(256) void k_region_scatter(
    int64_t R, int64_t n_seg, const int64_t *__restrict__ seg_off,
    const int64_t *__restrict__ slot, const int64_t *__restrict__ u_first, int64_t K_max,
    const double *__restrict__ dchi2, double *__restrict__ store)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    int64_t lo = 0, hi = n_seg - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (seg_off[mid] <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    store[slot[lo] * K_max + u_first[lo] + (r - seg_off[lo])] = dchi2[r];
}

// accepted[k][a] = dchi2_data[pts[k]] <= crit[k][a]
__global__ __launch_bounds__(256) void k_region_accept(int64_t n, int n_alpha,
                                                       const int64_t *__restrict__ pts,
                                                       const double *__restrict__ crit,
                                                       const double *__restrict__ dd,
                                                       uint8_t *__restrict__ accepted)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n_alpha) return;
    const int64_t k = e / n_alpha;
    accepted[e] = (dd[pts[k]] <= crit[e]) ? 1 : 0;
}

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes > 0 ? bytes : 16); }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

}  // namespace

// Scan one batch of generated universes (rows of d with true points p_idx)
// into dchi2 in the requested form.
static hipError_t scan_batch(const fc_grid *g, int form, int64_t R, const double *d,
                             const int64_t *p_idx, double *dchi2, double *chi2_min,
                             int64_t *argmin, double *chi2_p, hipStream_t st)
{
    if (form == FC_FORM_FP64) return launch_scan_fp64(g, R, d, p_idx, dchi2, chi2_min, argmin,
                                                      chi2_p, st);
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(chi2_min);
    hipError_t e = launch_init_keys(R, keys, chi2_p, st);
    if (e != hipSuccess) return e;
    if (form == FC_FORM_FP32)
        e = launch_scan_fp32(g, R, d, p_idx, 0, g->G, keys, chi2_p, st);
    else
        e = launch_scan_split(g, form == FC_FORM_SPLIT_FP16, R, d, p_idx, 0, g->G, keys, chi2_p,
                              st);
    if (e != hipSuccess) return e;
    return launch_finalize(R, p_idx, keys, chi2_min, argmin, chi2_p, dchi2, st);
}

int region_run(const fc_grid *g, int form, int64_t n_pts, const int64_t *pts_host, int64_t K0,
               int64_t K_max, double z, uint64_t seed, int n_alpha, const double *alpha,
               const double *dchi2_data, double *crit, uint8_t *accepted, int64_t *K_used,
               int32_t *n_rounds, double *n_evals, hipStream_t st, hipError_t *err)
{
    const int N = g->N;
    const int64_t G = g->G;
    // rows per batch: universes drawn and scanned together
    const int64_t R_max = int64_t(1) << 19;
    std::vector<int64_t> pts(n_pts);
    for (int64_t k = 0; k < n_pts; ++k) pts[k] = pts_host ? pts_host[k] : k;

    DevBuf store, d_pts, d_lo, d_hi, d_band, d_ranks, bd, bp, bkeys, barg, bcp, bdchi2, bseg, bslot,
        buf, bpts;
    hipError_t e;
    const int nq = 2 * n_alpha;
    const int64_t R_cap = std::min<int64_t>(R_max, n_pts * K_max);
    if ((e = store.alloc(sizeof(double) * (size_t)n_pts * K_max)) != hipSuccess ||
        (e = d_pts.alloc(sizeof(int64_t) * n_pts)) != hipSuccess ||
        (e = d_lo.alloc(sizeof(int64_t) * n_pts)) != hipSuccess ||
        (e = d_hi.alloc(sizeof(int64_t) * n_pts)) != hipSuccess ||
        (e = d_band.alloc(sizeof(double) * n_pts * nq)) != hipSuccess ||
        (e = d_ranks.alloc(sizeof(int64_t) * n_pts * nq)) != hipSuccess ||
        (e = bd.alloc(sizeof(double) * (size_t)R_cap * N)) != hipSuccess ||
        (e = bp.alloc(sizeof(int64_t) * R_cap)) != hipSuccess ||
        (e = bkeys.alloc(sizeof(double) * R_cap)) != hipSuccess ||
        (e = barg.alloc(sizeof(int64_t) * R_cap)) != hipSuccess ||
        (e = bcp.alloc(sizeof(double) * R_cap)) != hipSuccess ||
        (e = bdchi2.alloc(sizeof(double) * R_cap)) != hipSuccess ||
        (e = bseg.alloc(sizeof(int64_t) * (n_pts + 1))) != hipSuccess ||
        (e = bslot.alloc(sizeof(int64_t) * n_pts)) != hipSuccess ||
        (e = buf.alloc(sizeof(int64_t) * n_pts)) != hipSuccess ||
        (e = bpts.alloc(sizeof(int64_t) * n_pts)) != hipSuccess) {
        *err = e;
        return FC_ERR_NOMEM;
    }
    // the data's Delta chi^2 at every point, on the host for the decisions
    std::vector<double> dd_all(G), dd(n_pts);
    std::vector<int64_t> lo(n_pts), hi(n_pts);
    for (int64_t k = 0; k < n_pts; ++k) lo[k] = k * K_max;
    if ((e = hipMemcpyAsync(dd_all.data(), dchi2_data, sizeof(double) * G, hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(d_pts.p, pts.data(), sizeof(int64_t) * n_pts, hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(d_lo.p, lo.data(), sizeof(int64_t) * n_pts, hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        *err = e;
        return FC_ERR_DEVICE;
    }
    for (int64_t k = 0; k < n_pts; ++k) dd[k] = dd_all[pts[k]];

    std::vector<int64_t> K(n_pts, 0), K_new(n_pts, K0);
    std::vector<int64_t> b_seg, b_pt, b_uf, b_slot;
    std::vector<int64_t> ranks((size_t)n_pts * nq);
    std::vector<double> band((size_t)n_pts * nq);
    double evals = 0.0;
    int rounds = 0;
    for (;;) {
        // ---- draw and scan the new universes of this round, in batches ------
        int64_t k = 0, done_in_k = 0;
        bool any = false;
        while (k < n_pts) {
            b_seg.assign(1, 0);
            b_pt.clear();
            b_uf.clear();
            b_slot.clear();
            int64_t rows = 0;
            while (k < n_pts && rows < R_cap) {
                const int64_t need = K_new[k] - K[k] - done_in_k;
                if (need <= 0) {
                    ++k;
                    done_in_k = 0;
                    continue;
                }
                const int64_t take = std::min(need, R_cap - rows);
                b_pt.push_back(pts[k]);
                b_uf.push_back(K[k] + done_in_k);
                b_slot.push_back(k);
                rows += take;
                b_seg.push_back(rows);
                done_in_k += take;
                if (done_in_k == K_new[k] - K[k]) {
                    ++k;
                    done_in_k = 0;
                }
            }
            if (rows == 0) break;
            any = true;
            const int64_t nb = (int64_t)b_pt.size();
            if ((e = hipMemcpyAsync(bseg.p, b_seg.data(), sizeof(int64_t) * (nb + 1),
                                    hipMemcpyHostToDevice, st)) != hipSuccess ||
                (e = hipMemcpyAsync(bpts.p, b_pt.data(), sizeof(int64_t) * nb,
                                    hipMemcpyHostToDevice, st)) != hipSuccess ||
                (e = hipMemcpyAsync(buf.p, b_uf.data(), sizeof(int64_t) * nb,
                                    hipMemcpyHostToDevice, st)) != hipSuccess ||
                (e = hipMemcpyAsync(bslot.p, b_slot.data(), sizeof(int64_t) * nb,
                                    hipMemcpyHostToDevice, st)) != hipSuccess ||
                (e = launch_gen_universes(g, nb, bpts.as<int64_t>(), bseg.as<int64_t>(),
                                          buf.as<int64_t>(), seed, rows, bd.as<double>(),
                                          bp.as<int64_t>(), nullptr, st)) != hipSuccess ||
                (e = scan_batch(g, form, rows, bd.as<double>(), bp.as<int64_t>(),
                                bdchi2.as<double>(), bkeys.as<double>(), barg.as<int64_t>(),
                                bcp.as<double>(), st)) != hipSuccess) {
                *err = e;
                return FC_ERR_DEVICE;
            }
            hipLaunchKernelGGL(k_region_scatter, dim3((unsigned)((rows + 255) / 256)), dim3(256),
                               0, st, rows, nb, bseg.as<int64_t>(), bslot.as<int64_t>(),
                               buf.as<int64_t>(), K_max, bdchi2.as<double>(),
                               store.as<double>());
            if ((e = hipGetLastError()) != hipSuccess ||
                (e = hipStreamSynchronize(st)) != hipSuccess) {  // host batch arrays reused
                *err = e;
                return FC_ERR_DEVICE;
            }
            evals += (double)rows * (double)G;
        }
        if (!any) break;
        ++rounds;
        for (int64_t i = 0; i < n_pts; ++i) K[i] = K_new[i];

        // ---- critical values and bands over every point's K(p) values -------
        for (int64_t i = 0; i < n_pts; ++i) {
            hi[i] = lo[i] + K[i];
            for (int a = 0; a < n_alpha; ++a) {
                int64_t j = (int64_t)std::ceil(alpha[a] * (double)K[i]);
                j = std::min<int64_t>(std::max<int64_t>(j, 1), K[i]);
                const double var = (double)K[i] * alpha[a] * (1.0 - alpha[a]);
                const int64_t delta = (int64_t)std::ceil(z * std::sqrt(var));
                ranks[i * nq + 2 * a] = std::max<int64_t>(1, j - delta);
                ranks[i * nq + 2 * a + 1] = std::min<int64_t>(K[i], j + delta);
            }
        }
        if ((e = hipMemcpyAsync(d_hi.p, hi.data(), sizeof(int64_t) * n_pts, hipMemcpyHostToDevice,
                                st)) != hipSuccess ||
            (e = hipMemcpyAsync(d_ranks.p, ranks.data(), sizeof(int64_t) * n_pts * nq,
                                hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = launch_crit_gapped(n_pts, d_lo.as<int64_t>(), d_hi.as<int64_t>(),
                                    store.as<double>(), n_alpha, alpha, crit, st)) !=
                hipSuccess ||
            (e = launch_select_ranks(n_pts, d_lo.as<int64_t>(), d_hi.as<int64_t>(),
                                     store.as<double>(), nq, d_ranks.as<int64_t>(),
                                     d_band.as<double>(), st)) != hipSuccess ||
            (e = hipMemcpyAsync(band.data(), d_band.p, sizeof(double) * n_pts * nq,
                                hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess) {
            *err = e;
            return FC_ERR_DEVICE;
        }
        // ---- undecided points double their universes ------------------------
        for (int64_t i = 0; i < n_pts; ++i) {
            bool undecided = false;
            for (int a = 0; a < n_alpha; ++a)
                if (band[i * nq + 2 * a] <= dd[i] && dd[i] <= band[i * nq + 2 * a + 1])
                    undecided = true;
            K_new[i] = (undecided && K[i] < K_max) ? std::min(2 * K[i], K_max) : K[i];
        }
    }
    const int64_t ne = n_pts * n_alpha;
    hipLaunchKernelGGL(k_region_accept, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st,
                       n_pts, n_alpha, d_pts.as<int64_t>(), crit, dchi2_data, accepted);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(st)) != hipSuccess) {
        *err = e;
        return FC_ERR_DEVICE;
    }
    for (int64_t i = 0; i < n_pts; ++i) K_used[i] = K[i];
    *n_rounds = rounds;
    *n_evals = evals;
    return FC_OK;
}

}  // namespace fcx
