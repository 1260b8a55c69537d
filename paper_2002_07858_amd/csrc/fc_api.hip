// fc_api.hip -- host side of the C ABI declared in include/fc.h.
//
// Validation happens here, before any device work; every step of the path
// itself runs in the kernels of k_grid / k_cov / k_scan / k_crit.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "fc_internal.h"

#include <vector>

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? FC_ERR_NOMEM : FC_ERR_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define FC_HIP(call, what)                       \
    do {                                         \
        hipError_t e_ = (call);                  \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

void free_forms(fc_grid *g)
{
    if (g->W64) (void)hipFree(g->W64);
    if (g->R64) (void)hipFree(g->R64);
    if (g->R32) (void)hipFree(g->R32);
    if (g->RB16) (void)hipFree(g->RB16);
    if (g->RH16) (void)hipFree(g->RH16);
    if (g->F64) (void)hipFree(g->F64);
    if (g->LF64) (void)hipFree(g->LF64);
    g->W64 = nullptr;
    g->R64 = nullptr;
    g->R32 = nullptr;
    g->RB16 = nullptr;
    g->RH16 = nullptr;
    g->F64 = nullptr;
    g->LF64 = nullptr;
    g->lf_ok = 0;
    g->forms = 0;
}

size_t split_record_bytes(const fc_grid *g)
{
    return sizeof(uint4) * (size_t)fcx::split_rec_units(g->N);
}

size_t grid_bytes(const fc_grid *g)
{
    size_t b = 0;
    b += sizeof(double) * (size_t)g->G * g->N;  // S64
    if (g->W64) b += sizeof(double) * (size_t)g->G * ((size_t)g->N * (g->N + 1) / 2);
    if (g->R64) b += sizeof(uint4) * (size_t)g->G * fcx::f64_rec_units(g->N);
    b += sizeof(double) * 128;                  // off, dev
    if (g->R32) b += sizeof(uint4) * (size_t)g->G * fcx::rec_units(g->ns);
    if (g->RB16) b += (size_t)g->G * split_record_bytes(g);
    if (g->RH16) b += (size_t)g->G * split_record_bytes(g);
    if (g->F64) b += 2 * sizeof(double) * (size_t)g->N * g->N;  // F and its factor
    return b;
}

bool finite_all(const double *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return false;
    return true;
}

}  // namespace

namespace fcx {
// Record a failure for fc_last_error on the calling thread; returns code.
int set_last_error(int code, const char *msg)
{
    g_last_error = msg;
    return code;
}
}  // namespace fcx

extern "C" {

const char *fc_last_error(void) { return g_last_error.c_str(); }

int fc_build_grid(fc_grid **out, int32_t D, const int64_t *axis_len, const double *axis_vals,
                  int32_t N, const double *signal, const double *central, hipStream_t stream)
{
    g_last_error.clear();
    if (!out) return fail(FC_ERR_INVALID_ARG, "fc_build_grid: out is NULL");
    *out = nullptr;
    if (D < 1 || D > 16) return fail(FC_ERR_INVALID_ARG, "fc_build_grid: D=%d not in 1..16", D);
    if (!axis_len || !axis_vals || !signal)
        return fail(FC_ERR_INVALID_ARG, "fc_build_grid: NULL axis_len/axis_vals/signal");
    if (N < 1) return fail(FC_ERR_INVALID_ARG, "fc_build_grid: N=%d < 1", N);
    if (N > FC_MAX_BINS)
        return fail(FC_ERR_UNSUPPORTED, "fc_build_grid: N=%d > %d bins", N, FC_MAX_BINS);
    int64_t G = 1, nvals = 0;
    for (int32_t e = 0; e < D; ++e) {
        if (axis_len[e] < 1)
            return fail(FC_ERR_INVALID_ARG, "fc_build_grid: axis %d has length %lld", e,
                        (long long)axis_len[e]);
        if (G > (int64_t(1) << 31) / axis_len[e])
            return fail(FC_ERR_INVALID_ARG, "fc_build_grid: grid has >= 2^31 points");
        G *= axis_len[e];
        nvals += axis_len[e];
    }
    if (G >= (int64_t(1) << 31)) return fail(FC_ERR_INVALID_ARG, "fc_build_grid: grid too large");
    if (!finite_all(signal, (size_t)G * N))
        return fail(FC_ERR_INVALID_ARG, "fc_build_grid: signal has a non-finite entry");

    fc_grid *g = new (std::nothrow) fc_grid();
    if (!g) return fail(FC_ERR_NOMEM, "fc_build_grid: host allocation failed");
    g->D = D;
    g->N = N;
    g->G = G;
    g->axis_len.assign(axis_len, axis_len + D);
    g->axis_vals.assign(axis_vals, axis_vals + nvals);
    if (central) g->central.assign(central, central + N);
    g->ns = fcx::n_ksteps(N);
    g->ng = fcx::n_groups_from_ns(g->ns);
    (void)hipGetDevice(&g->device);

    hipError_t e;
    if ((e = hipMalloc(&g->S64, sizeof(double) * (size_t)G * N)) != hipSuccess ||
        (e = hipMalloc(&g->off, sizeof(double) * 64)) != hipSuccess ||
        (e = hipMalloc(&g->dev, sizeof(double) * 64)) != hipSuccess) {
        fc_grid_destroy(g);
        return hip_fail(e, "fc_build_grid: hipMalloc");
    }
    double hdev[64];
    if ((e = hipMemcpyAsync(g->S64, signal, sizeof(double) * (size_t)G * N, hipMemcpyHostToDevice,
                            stream)) != hipSuccess ||
        (e = fcx::launch_offset(g->S64, G, N, g->off, g->dev, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(hdev, g->dev, sizeof(hdev), hipMemcpyDeviceToHost, stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
        fc_grid_destroy(g);
        return hip_fail(e, "fc_build_grid: upload/stage");
    }
    // split-FP16 range: 2^ed16 max|S - o| < 2^13
    double dmax = 0.0;
    for (int j = 0; j < N; ++j) dmax = fmax(dmax, hdev[j]);
    g->ed16 = (dmax > 0.0) ? 12 - ilogb(dmax) : 0;
    g->bytes = grid_bytes(g);
    *out = g;
    return FC_OK;
}

int fc_build_covariance(fc_grid *g, const double *frac_cov, int32_t stat_mode,
                        const double *stat_diag, uint32_t forms, int64_t *bad_q,
                        hipStream_t stream)
{
    g_last_error.clear();
    if (bad_q) *bad_q = -1;
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_build_covariance: grid is NULL");
    if (!frac_cov || !bad_q) return fail(FC_ERR_INVALID_ARG, "fc_build_covariance: NULL argument");
    if (stat_mode != FC_STAT_PEARSON && stat_mode != FC_STAT_FIXED)
        return fail(FC_ERR_INVALID_ARG, "fc_build_covariance: bad stat_mode %d", stat_mode);
    if (stat_mode == FC_STAT_FIXED && !stat_diag)
        return fail(FC_ERR_INVALID_ARG, "fc_build_covariance: FIXED mode needs stat_diag");
    const uint32_t known = FC_FORM_FP64 | FC_FORM_FP32 | FC_FORM_SPLIT_BF16 | FC_FORM_SPLIT_FP16;
    if (forms == 0 || (forms & ~known))
        return fail(FC_ERR_INVALID_ARG, "fc_build_covariance: bad forms mask 0x%x", forms);
    const int N = g->N;
    if (!finite_all(frac_cov, (size_t)N * N))
        return fail(FC_ERR_INVALID_ARG, "fc_build_covariance: frac_cov has a non-finite entry");
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < i; ++j)
            if (frac_cov[i * N + j] != frac_cov[j * N + i])
                return fail(FC_ERR_INVALID_ARG, "fc_build_covariance: frac_cov not symmetric");
    if (stat_mode == FC_STAT_FIXED && !finite_all(stat_diag, (size_t)N))
        return fail(FC_ERR_INVALID_ARG, "fc_build_covariance: stat_diag has a non-finite entry");

    free_forms(g);
    double *dF = nullptr, *dstat = nullptr, *dLF = nullptr;
    unsigned long long *dbad = nullptr;
    double *W64 = nullptr;
    uint4 *R64 = nullptr, *R32 = nullptr, *RB16 = nullptr, *RH16 = nullptr;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        if (dF) (void)hipFree(dF);
        if (dLF) (void)hipFree(dLF);
        if (dstat) (void)hipFree(dstat);
        if (dbad) (void)hipFree(dbad);
    };
    const size_t nt = (size_t)N * (N + 1) / 2;
    // gather maps of the record writers (depend on N only)
    std::vector<int16_t> hmaps(fcx::cov_maps_size(N, g->ns));
    fcx::cov_maps_fill(N, g->ns, hmaps.data());
    int16_t *dmaps = nullptr;
    if ((e = hipMalloc(&dmaps, sizeof(int16_t) * hmaps.size())) != hipSuccess)
        return hip_fail(e, "fc_build_covariance: hipMalloc");
    struct MapsGuard {
        int16_t *p;
        ~MapsGuard() { if (p) (void)hipFree(p); }
    } maps_guard{dmaps};
    if ((e = hipMalloc(&dF, sizeof(double) * N * N)) != hipSuccess ||
        (e = hipMalloc(&dLF, sizeof(double) * N * N)) != hipSuccess ||
        (e = hipMalloc(&dstat, sizeof(double) * N)) != hipSuccess ||
        (e = hipMalloc(&dbad, sizeof(unsigned long long))) != hipSuccess ||
        ((forms & FC_FORM_FP64) &&
         (e = hipMalloc(&W64, sizeof(double) * (size_t)g->G * nt)) != hipSuccess) ||
        ((forms & FC_FORM_FP64) &&
         (e = hipMalloc(&R64, sizeof(uint4) * (size_t)g->G *
                                  fcx::f64_rec_units(N))) != hipSuccess) ||
        ((forms & FC_FORM_FP32) &&
         (e = hipMalloc(&R32, sizeof(uint4) * (size_t)g->G * fcx::rec_units(g->ns))) !=
             hipSuccess) ||
        ((forms & FC_FORM_SPLIT_BF16) &&
         (e = hipMalloc(&RB16, (size_t)g->G * split_record_bytes(g))) != hipSuccess) ||
        ((forms & FC_FORM_SPLIT_FP16) &&
         (e = hipMalloc(&RH16, (size_t)g->G * split_record_bytes(g))) != hipSuccess)) {
        cleanup();
        if (W64) (void)hipFree(W64);
        if (R64) (void)hipFree(R64);
        if (R32) (void)hipFree(R32);
        if (RB16) (void)hipFree(RB16);
        if (RH16) (void)hipFree(RH16);
        return hip_fail(e, "fc_build_covariance: hipMalloc");
    }
    const unsigned long long none = ~0ull;
    unsigned long long hbad = none, hlf = 0;
    if ((e = hipMemcpyAsync(dmaps, hmaps.data(), sizeof(int16_t) * hmaps.size(),
                            hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(dF, frac_cov, sizeof(double) * N * N, hipMemcpyHostToDevice,
                            stream)) != hipSuccess ||
        (stat_mode == FC_STAT_FIXED &&
         (e = hipMemcpyAsync(dstat, stat_diag, sizeof(double) * N, hipMemcpyHostToDevice,
                             stream)) != hipSuccess) ||
        (e = hipMemcpyAsync(dbad, &none, sizeof(none), hipMemcpyHostToDevice, stream)) !=
            hipSuccess ||
        (e = fcx::launch_cov_build(g, dF, dstat, stat_mode, forms, dmaps, W64, R64, R32, RB16,
                                   RH16, dbad, stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&hbad, dbad, sizeof(hbad), hipMemcpyDeviceToHost, stream)) !=
            hipSuccess ||
        // the factor of F itself, for drawing universes (dbad reused as the flag)
        (e = fcx::launch_chol_frac(dF, N, dLF, reinterpret_cast<int *>(dbad), stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&hlf, dbad, sizeof(int), hipMemcpyDeviceToHost, stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
        cleanup();
        if (W64) (void)hipFree(W64);
        if (R64) (void)hipFree(R64);
        if (R32) (void)hipFree(R32);
        if (RB16) (void)hipFree(RB16);
        if (RH16) (void)hipFree(RH16);
        return hip_fail(e, "fc_build_covariance: build");
    }
    if (hbad != none) {
        cleanup();
        if (W64) (void)hipFree(W64);
        if (R64) (void)hipFree(R64);
        if (R32) (void)hipFree(R32);
        if (RB16) (void)hipFree(RB16);
        if (RH16) (void)hipFree(RH16);
        *bad_q = (int64_t)hbad;
        g->bytes = grid_bytes(g);
        return fail(FC_ERR_NOT_PD, "fc_build_covariance: covariance not positive definite at q=%lld",
                    (long long)hbad);
    }
    g->W64 = W64;
    g->R64 = R64;
    g->R32 = R32;
    g->RB16 = RB16;
    g->RH16 = RH16;
    g->F64 = dF;
    g->LF64 = dLF;
    g->lf_ok = ((int)hlf == 1) ? 1 : 0;
    dF = dLF = nullptr;  // kept on the grid
    cleanup();
    g->forms = forms;
    g->bytes = grid_bytes(g);
    return FC_OK;
}

}  // extern "C"

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Scratch memory of one scan call: stream-ordered allocations freed at the
// end of the call (in stream order), or pieces of a fixed region owned by
// someone else.
struct Scratch {
    hipStream_t st = nullptr;
    char *base = nullptr;  // fixed region, or nullptr for stream-ordered allocations
    size_t bytes = 0, used = 0;
    std::vector<void *> owned;

    hipError_t take(size_t n, void **out)
    {
        n = align256(n);
        if (base) {
            if (n > bytes - used) return hipErrorOutOfMemory;
            *out = base + used;
            used += n;
            return hipSuccess;
        }
        const hipError_t e = hipMallocAsync(out, n, st);
        if (e == hipSuccess) owned.push_back(*out);
        return e;
    }
    // what is left of a fixed region (nullptr, 0 for stream-ordered scratch)
    void *rest(size_t *n) const
    {
        *n = base ? bytes - used : 0;
        return base ? base + used : nullptr;
    }
    hipError_t release()
    {
        hipError_t e = hipSuccess;
        for (void *p : owned) {
            const hipError_t ef = hipFreeAsync(p, st);
            if (e == hipSuccess) e = ef;
        }
        owned.clear();
        return e;
    }
};

bool valid_form(int32_t form)
{
    return form == FC_FORM_FP64 || form == FC_FORM_FP32 || form == FC_FORM_SPLIT_BF16 ||
           form == FC_FORM_SPLIT_FP16;
}

// The scan of fc_scan once the arguments are checked: chi2_min, argmin and
// chi2_p may be nullptr (the keys and chi2_p then live in scratch).
int scan_checked(const char *fn, const fc_grid *g, int32_t form, int64_t K, const double *d,
                 const int64_t *p_idx, double *dchi2, double *chi2_min, int64_t *argmin,
                 double *chi2_p, hipStream_t stream, Scratch &sc)
{
    hipError_t e = hipSuccess;
    double *cp = chi2_p;
    if (!cp && (e = sc.take(sizeof(double) * (size_t)K, reinterpret_cast<void **>(&cp))) !=
                   hipSuccess)
        goto fail_alloc;
    if (form == FC_FORM_FP64) {
        size_t rest = 0;
        void *r = sc.rest(&rest);
        if ((e = fcx::launch_scan_fp64(g, K, d, p_idx, dchi2, chi2_min, argmin, cp, stream,
                                       static_cast<fcx::Fp64Part *>(r), rest)) != hipSuccess) {
            (void)sc.release();
            return hip_fail(e, fn);
        }
    } else {
        unsigned long long *keys = reinterpret_cast<unsigned long long *>(chi2_min);
        if (!keys && (e = sc.take(sizeof(uint64_t) * (size_t)K,
                                  reinterpret_cast<void **>(&keys))) != hipSuccess)
            goto fail_alloc;
        if ((e = fcx::launch_init_keys(K, keys, cp, stream)) != hipSuccess ||
            (e = (form == FC_FORM_FP32)
                     ? fcx::launch_scan_fp32(g, K, d, p_idx, 0, g->G, keys, cp, stream)
                     : fcx::launch_scan_split(g, form == FC_FORM_SPLIT_FP16, K, d, p_idx, 0,
                                              g->G, keys, cp, stream)) != hipSuccess ||
            (e = fcx::launch_finalize(K, p_idx, keys, chi2_min, argmin, cp, dchi2, stream)) !=
                hipSuccess) {
            (void)sc.release();
            return hip_fail(e, fn);
        }
    }
    if ((e = sc.release()) != hipSuccess) return hip_fail(e, fn);
    return FC_OK;
fail_alloc:
    (void)sc.release();
    if (sc.base)
        return fail(FC_ERR_INVALID_ARG, "%s: K=%lld needs more than the %zu bytes of scratch", fn,
                    (long long)K, sc.bytes);
    return hip_fail(e, fn);
}

// Argument checks of fc_scan (and its no-allocation variant).
int check_scan(const char *fn, const fc_grid *g, int32_t form, int64_t K, const double *d,
               const int64_t *p_idx, const double *dchi2)
{
    if (!g) return fail(FC_ERR_INVALID_ARG, "%s: grid is NULL", fn);
    if (!valid_form(form)) return fail(FC_ERR_INVALID_ARG, "%s: bad form %d", fn, form);
    if (!(g->forms & (uint32_t)form))
        return fail(FC_ERR_STATE, "%s: form %d was not built for this grid", fn, form);
    if (K < 0) return fail(FC_ERR_INVALID_ARG, "%s: K=%lld < 0", fn, (long long)K);
    if (K > (int64_t(1) << 30))
        return fail(FC_ERR_INVALID_ARG, "%s: K=%lld > 2^30 universes per call", fn, (long long)K);
    if (K > 0 && (!d || !p_idx || !dchi2))
        return fail(FC_ERR_INVALID_ARG, "%s: NULL d, p_idx or dchi2", fn);
    return FC_OK;
}

// Static scratch of fc_scan_no_alloc: one array per device (each device that
// loads the library holds its own copy until the process ends).  In host code
// `scratch` names a host-side stand-in, never the device memory: the device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is passed to kernels.
__device__ __align__(256) unsigned char scratch[FC_NO_ALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

hipError_t static_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = a;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int fc_scan_no_alloc(const fc_grid *g, int32_t form, int64_t K, const double *d,
                     const int64_t *p_idx, double *dchi2, double *chi2_min, int64_t *argmin,
                     double *chi2_p, hipStream_t stream)
{
    g_last_error.clear();
    const int rc = check_scan("fc_scan_no_alloc", g, form, K, d, p_idx, dchi2);
    if (rc != FC_OK || K == 0) return rc;
    void *base = nullptr;
    const hipError_t e = static_scratch(&base);
    if (e != hipSuccess) return hip_fail(e, "fc_scan_no_alloc: static scratch address");
    Scratch sc;
    sc.st = stream;
    sc.base = static_cast<char *>(base);
    sc.bytes = FC_NO_ALLOC_SCRATCH_BYTES;
    return scan_checked("fc_scan_no_alloc", g, form, K, d, p_idx, dchi2, chi2_min, argmin, chi2_p,
                        stream, sc);
}

int fc_scan(const fc_grid *g, int32_t form, int64_t K, const double *d, const int64_t *p_idx,
            double *dchi2, double *chi2_min, int64_t *argmin, double *chi2_p, hipStream_t stream)
{
    g_last_error.clear();
    const int rc = check_scan("fc_scan", g, form, K, d, p_idx, dchi2);
    if (rc != FC_OK || K == 0) return rc;
    Scratch sc;
    sc.st = stream;
    return scan_checked("fc_scan", g, form, K, d, p_idx, dchi2, chi2_min, argmin, chi2_p, stream,
                        sc);
}

namespace {

// Workspace of a points scan over nq grid points: p_idx [K] int64 and, for
// the FP32 form, the tile prefix [n_pts+1] int64 and the offset table
// [n_pts][nq][4 ns] FP32.
size_t points_workspace(const fc_grid *g, int32_t form, int64_t n_pts, int64_t K, int64_t nq)
{
    // a size past 2^60 bytes (no device holds it) is reported as SIZE_MAX
    // rather than wrapped around
    const double table =
        (form == FC_FORM_FP32) ? 4.0 * (double)n_pts * (double)nq * 4.0 * (double)g->ns : 0.0;
    if (8.0 * (double)K + table > 1.152921504606847e18) return SIZE_MAX;
    size_t b = align256(sizeof(int64_t) * (size_t)K);
    if (form == FC_FORM_FP32)
        b += align256(sizeof(int64_t) * (size_t)(n_pts + 1)) +
             sizeof(float) * (size_t)n_pts * (size_t)nq * 4 * (size_t)g->ns;
    return b;
}

struct PointsWs {
    int64_t *p_idx;
    int64_t *tile_start;
    float *T;
};

PointsWs carve_points_ws(void *workspace, int64_t n_pts, int64_t K)
{
    char *ws = static_cast<char *>(workspace);
    PointsWs w;
    w.p_idx = reinterpret_cast<int64_t *>(ws);
    w.tile_start = reinterpret_cast<int64_t *>(ws + align256(sizeof(int64_t) * (size_t)K));
    w.T = reinterpret_cast<float *>(ws + align256(sizeof(int64_t) * (size_t)K) +
                                    align256(sizeof(int64_t) * (size_t)(n_pts + 1)));
    return w;
}

}  // namespace

int fc_scan_points_workspace(const fc_grid *g, int32_t form, int64_t n_pts, int64_t K,
                             size_t *bytes)
{
    g_last_error.clear();
    if (!g || !bytes) return fail(FC_ERR_INVALID_ARG, "fc_scan_points_workspace: NULL argument");
    if (n_pts < 0 || K < 0 || n_pts > 0x7fffffff)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_workspace: bad n_pts or K");
    *bytes = points_workspace(g, form, n_pts, K, g->G);
    if (*bytes == SIZE_MAX)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_workspace: size beyond 2^60 bytes");
    return FC_OK;
}

int fc_scan_points(const fc_grid *g, int32_t form, int64_t n_pts, const int64_t *p,
                   const int64_t *seg_off, int64_t K, const double *d, void *workspace,
                   size_t workspace_bytes, double *dchi2, double *chi2_min, int64_t *argmin,
                   double *chi2_p, hipStream_t stream)
{
    g_last_error.clear();
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_scan_points: grid is NULL");
    if (form != FC_FORM_FP64 && form != FC_FORM_FP32 && form != FC_FORM_SPLIT_BF16 &&
        form != FC_FORM_SPLIT_FP16)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points: bad form %d", form);
    if (!(g->forms & (uint32_t)form))
        return fail(FC_ERR_STATE, "fc_scan_points: form %d was not built for this grid", form);
    if (K < 0 || n_pts < 0 || n_pts > 0x7fffffff)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points: bad n_pts or K");
    if (K == 0) return FC_OK;
    if (n_pts == 0) return fail(FC_ERR_INVALID_ARG, "fc_scan_points: K > 0 universes, no points");
    if (K > (int64_t(1) << 30))
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points: K=%lld > 2^30", (long long)K);
    if (!p || !seg_off || !d || !workspace || !dchi2)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points: NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points: workspace not 256-byte aligned");
    const size_t need = points_workspace(g, form, n_pts, K, g->G);
    if (need == SIZE_MAX || workspace_bytes < need)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points: workspace %zu B < %zu B", workspace_bytes,
                    need);
    const PointsWs w = carve_points_ws(workspace, n_pts, K);
    hipError_t e;
    if ((e = fcx::launch_expand_segments(K, n_pts, seg_off, p, w.p_idx, stream)) != hipSuccess)
        return hip_fail(e, "fc_scan_points: segment expansion");
    Scratch sc;
    sc.st = stream;
    if (form != FC_FORM_FP32)
        return scan_checked("fc_scan_points", g, form, K, d, w.p_idx, dchi2, chi2_min, argmin,
                            chi2_p, stream, sc);
    double *cp = chi2_p;
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(chi2_min);
    if ((!cp && (e = sc.take(sizeof(double) * (size_t)K, reinterpret_cast<void **>(&cp))) !=
                    hipSuccess) ||
        (!keys && (e = sc.take(sizeof(uint64_t) * (size_t)K, reinterpret_cast<void **>(&keys))) !=
                      hipSuccess)) {
        (void)sc.release();
        return hip_fail(e, "fc_scan_points: scratch");
    }
    if ((e = fcx::launch_offset_table(g, n_pts, p, 0, g->G, w.T, stream)) != hipSuccess ||
        (e = fcx::launch_init_keys(K, keys, cp, stream)) != hipSuccess ||
        (e = fcx::launch_scan_fp32_points(g, n_pts, p, seg_off, K, d, 0, g->G, w.T, w.tile_start,
                                          keys, cp, stream)) != hipSuccess ||
        (e = fcx::launch_finalize(K, w.p_idx, keys, chi2_min, argmin, cp, dchi2, stream)) !=
            hipSuccess) {
        (void)sc.release();
        return hip_fail(e, "fc_scan_points: fp32 launch");
    }
    if ((e = sc.release()) != hipSuccess) return hip_fail(e, "fc_scan_points: scratch");
    return FC_OK;
}

// ---- grid-sliced scans ------------------------------------------------------

int fc_scan_state_init(int64_t K, uint64_t *keys, double *chi2_p, hipStream_t stream)
{
    g_last_error.clear();
    if (K < 0 || K > (int64_t(1) << 30))
        return fail(FC_ERR_INVALID_ARG, "fc_scan_state_init: K=%lld out of [0, 2^30]",
                    (long long)K);
    if (K == 0) return FC_OK;
    if (!keys || !chi2_p) return fail(FC_ERR_INVALID_ARG, "fc_scan_state_init: NULL pointer");
    const hipError_t e = fcx::launch_init_keys(K, reinterpret_cast<unsigned long long *>(keys),
                                               chi2_p, stream, 0.0);
    if (e != hipSuccess) return hip_fail(e, "fc_scan_state_init: launch");
    return FC_OK;
}

namespace {

// Checks shared by the two slice entry points: FC_OK, or the error (message set).
int check_slice(const char *fn, const fc_grid *g, int32_t form, int64_t K, int64_t q0, int64_t nq)
{
    if (!g) return fail(FC_ERR_INVALID_ARG, "%s: grid is NULL", fn);
    if (form != FC_FORM_FP64 && form != FC_FORM_FP32 && form != FC_FORM_SPLIT_BF16 &&
        form != FC_FORM_SPLIT_FP16)
        return fail(FC_ERR_INVALID_ARG, "%s: bad form %d", fn, form);
    if (form == FC_FORM_FP64)
        return fail(FC_ERR_UNSUPPORTED,
                    "%s: the FP64 form keeps FP64 minima, which a 64-bit key cannot merge", fn);
    if (!(g->forms & (uint32_t)form))
        return fail(FC_ERR_STATE, "%s: form %d was not built for this grid", fn, form);
    if (K < 0 || K > (int64_t(1) << 30))
        return fail(FC_ERR_INVALID_ARG, "%s: K=%lld out of [0, 2^30]", fn, (long long)K);
    if (q0 < 0 || nq < 0 || q0 > g->G || nq > g->G - q0)
        return fail(FC_ERR_INVALID_ARG, "%s: grid slice [%lld, %lld) outside [0, %lld)", fn,
                    (long long)q0, (long long)(q0 + nq), (long long)g->G);
    return FC_OK;
}

}  // namespace

int fc_scan_slice(const fc_grid *g, int32_t form, int64_t K, const double *d, const int64_t *p_idx,
                  int64_t q0, int64_t nq, uint64_t *keys, double *chi2_p, hipStream_t stream)
{
    g_last_error.clear();
    int rc = check_slice("fc_scan_slice", g, form, K, q0, nq);
    if (rc != FC_OK) return rc;
    if (K == 0 || nq == 0) return FC_OK;
    if (!d || !p_idx || !keys || !chi2_p)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_slice: NULL device pointer");
    unsigned long long *k = reinterpret_cast<unsigned long long *>(keys);
    const hipError_t e =
        form == FC_FORM_FP32
            ? fcx::launch_scan_fp32(g, K, d, p_idx, q0, nq, k, chi2_p, stream)
            : fcx::launch_scan_split(g, form == FC_FORM_SPLIT_FP16, K, d, p_idx, q0, nq, k, chi2_p,
                                     stream);
    if (e != hipSuccess) return hip_fail(e, "fc_scan_slice: launch");
    return FC_OK;
}

int fc_scan_points_slice_workspace(const fc_grid *g, int32_t form, int64_t n_pts, int64_t K,
                                   int64_t nq, size_t *bytes)
{
    g_last_error.clear();
    if (!g || !bytes)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_slice_workspace: NULL argument");
    if (n_pts < 0 || K < 0 || n_pts > 0x7fffffff || nq < 0 || nq > g->G)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_slice_workspace: bad n_pts, K or nq");
    *bytes = points_workspace(g, form, n_pts, K, nq);
    if (*bytes == SIZE_MAX)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_slice_workspace: size beyond 2^60 bytes");
    return FC_OK;
}

int fc_scan_points_slice(const fc_grid *g, int32_t form, int64_t n_pts, const int64_t *p,
                         const int64_t *seg_off, int64_t K, const double *d, int64_t q0,
                         int64_t nq, void *workspace, size_t workspace_bytes, uint64_t *keys,
                         double *chi2_p, hipStream_t stream)
{
    g_last_error.clear();
    int rc = check_slice("fc_scan_points_slice", g, form, K, q0, nq);
    if (rc != FC_OK) return rc;
    if (n_pts < 0 || n_pts > 0x7fffffff)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_slice: bad n_pts");
    if (K == 0 || nq == 0) return FC_OK;
    if (n_pts == 0)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_slice: K > 0 universes, no points");
    if (!p || !seg_off || !d || !workspace || !keys || !chi2_p)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_slice: NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_slice: workspace not 256-byte aligned");
    const size_t need = points_workspace(g, form, n_pts, K, nq);
    if (need == SIZE_MAX || workspace_bytes < need)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_points_slice: workspace %zu B < %zu B",
                    workspace_bytes, need);
    const PointsWs w = carve_points_ws(workspace, n_pts, K);
    unsigned long long *k = reinterpret_cast<unsigned long long *>(keys);
    hipError_t e;
    if (form != FC_FORM_FP32) {
        if ((e = fcx::launch_expand_segments(K, n_pts, seg_off, p, w.p_idx, stream)) !=
                hipSuccess ||
            (e = fcx::launch_scan_split(g, form == FC_FORM_SPLIT_FP16, K, d, w.p_idx, q0, nq, k,
                                        chi2_p, stream)) != hipSuccess)
            return hip_fail(e, "fc_scan_points_slice: split launch");
        return FC_OK;
    }
    if ((e = fcx::launch_offset_table(g, n_pts, p, q0, nq, w.T, stream)) != hipSuccess ||
        (e = fcx::launch_scan_fp32_points(g, n_pts, p, seg_off, K, d, q0, nq, w.T, w.tile_start,
                                          k, chi2_p, stream)) != hipSuccess)
        return hip_fail(e, "fc_scan_points_slice: fp32 launch");
    return FC_OK;
}

int fc_scan_state_finalize(const fc_grid *g, int64_t K, const int64_t *p_idx,
                           const uint64_t *keys, const double *chi2_p, double *dchi2,
                           double *chi2_min, int64_t *argmin, hipStream_t stream)
{
    g_last_error.clear();
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_scan_state_finalize: grid is NULL");
    if (K < 0 || K > (int64_t(1) << 30))
        return fail(FC_ERR_INVALID_ARG, "fc_scan_state_finalize: K=%lld out of [0, 2^30]",
                    (long long)K);
    if (K == 0) return FC_OK;
    if (!p_idx || !keys || !chi2_p || !dchi2 || !chi2_min || !argmin)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_state_finalize: NULL device pointer");
    const hipError_t e =
        fcx::launch_finalize(K, p_idx, reinterpret_cast<const unsigned long long *>(keys),
                             chi2_min, argmin, chi2_p, dchi2, stream, -1, g->G);
    if (e != hipSuccess) return hip_fail(e, "fc_scan_state_finalize: launch");
    return FC_OK;
}

int fc_critical_value(int64_t n_seg, const int64_t *seg_off, const double *dchi2, int32_t n_alpha,
                      const double *alpha, double *crit, int32_t n_bins, double hist_hi,
                      int64_t *hist, hipStream_t stream)
{
    g_last_error.clear();
    if (n_seg < 0) return fail(FC_ERR_INVALID_ARG, "fc_critical_value: n_seg < 0");
    if (n_seg > 0x7fffffff) return fail(FC_ERR_INVALID_ARG, "fc_critical_value: n_seg too large");
    if (n_alpha < 1 || n_alpha > 8)
        return fail(FC_ERR_INVALID_ARG, "fc_critical_value: n_alpha=%d not in 1..8", n_alpha);
    if (!alpha) return fail(FC_ERR_INVALID_ARG, "fc_critical_value: alpha is NULL");
    for (int a = 0; a < n_alpha; ++a)
        if (!(alpha[a] > 0.0 && alpha[a] <= 1.0))
            return fail(FC_ERR_INVALID_ARG, "fc_critical_value: alpha[%d]=%g not in (0,1]", a,
                        alpha[a]);
    if (hist) {
        if (n_bins < 1 || n_bins > 16383)
            return fail(FC_ERR_INVALID_ARG, "fc_critical_value: n_bins=%d not in 1..16383", n_bins);
        if (!(hist_hi > 0.0) || !isfinite(hist_hi))
            return fail(FC_ERR_INVALID_ARG, "fc_critical_value: hist_hi must be finite and > 0");
    }
    if (n_seg == 0) return FC_OK;
    if (!seg_off || !dchi2 || !crit)
        return fail(FC_ERR_INVALID_ARG, "fc_critical_value: NULL device pointer");
    hipError_t e = fcx::launch_crit(n_seg, seg_off, dchi2, n_alpha, alpha, crit, n_bins, hist_hi,
                                    hist, stream);
    if (e != hipSuccess) return hip_fail(e, "fc_critical_value: launch");
    return FC_OK;
}

int fc_data_scan(const fc_grid *g, const double *central, double *dchi2_data, double *chi2_min,
                 int64_t *argmin, hipStream_t stream)
{
    g_last_error.clear();
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_data_scan: grid is NULL");
    if (!dchi2_data || !chi2_min || !argmin)
        return fail(FC_ERR_INVALID_ARG, "fc_data_scan: NULL output");
    if (!(g->forms & FC_FORM_FP64)) return fail(FC_ERR_STATE, "fc_data_scan: FP64 form not built");
    const double *c = central ? central : (g->central.empty() ? nullptr : g->central.data());
    if (!c) return fail(FC_ERR_STATE, "fc_data_scan: no central data vector");
    double *dc = nullptr;
    unsigned long long *scratch = nullptr;
    unsigned long long hs[2] = {0, 0};
    hipError_t e;
    if ((e = hipMalloc(&dc, sizeof(double) * g->N)) != hipSuccess ||
        (e = hipMalloc(&scratch, sizeof(unsigned long long) * 2)) != hipSuccess ||
        (e = hipMemcpyAsync(dc, c, sizeof(double) * g->N, hipMemcpyHostToDevice, stream)) !=
            hipSuccess ||
        (e = fcx::launch_data_scan(g, dc, dchi2_data, scratch, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(hs, scratch, sizeof(hs), hipMemcpyDeviceToHost, stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
        if (dc) (void)hipFree(dc);
        if (scratch) (void)hipFree(scratch);
        return hip_fail(e, "fc_data_scan");
    }
    (void)hipFree(dc);
    (void)hipFree(scratch);
    // decode the ordered key of the minimum
    if (hs[0] == ~0ull) {
        *chi2_min = NAN;
        *argmin = -1;
    } else {
        const unsigned long long b = (hs[0] >> 63) ? (hs[0] & 0x7fffffffffffffffull) : ~hs[0];
        double v;
        memcpy(&v, &b, sizeof(v));
        *chi2_min = v;
        *argmin = (int64_t)hs[1];
    }
    return FC_OK;
}

int fc_acceptance(const fc_grid *g, int64_t n_pts, const int64_t *p, const double *crit,
                  int64_t crit_stride, const double *dchi2_data, uint8_t *accepted,
                  hipStream_t stream)
{
    g_last_error.clear();
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_acceptance: grid is NULL");
    if (n_pts < 0 || crit_stride < 1)
        return fail(FC_ERR_INVALID_ARG, "fc_acceptance: bad n_pts or crit_stride");
    if (n_pts == 0) return FC_OK;
    if (!p || !crit || !dchi2_data || !accepted)
        return fail(FC_ERR_INVALID_ARG, "fc_acceptance: NULL device pointer");
    hipError_t e = fcx::launch_accept(n_pts, p, crit, crit_stride, dchi2_data, g->G, accepted,
                                      stream);
    if (e != hipSuccess) return hip_fail(e, "fc_acceptance");
    return FC_OK;
}

int fc_generate_universes(const fc_grid *g, int64_t n_pts, const int64_t *p,
                          const int64_t *seg_off, const int64_t *u_first, uint64_t seed,
                          int64_t K, double *d, int64_t *p_idx, int32_t *counts,
                          hipStream_t stream)
{
    g_last_error.clear();
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_generate_universes: grid is NULL");
    if (n_pts < 0 || K < 0) return fail(FC_ERR_INVALID_ARG, "fc_generate_universes: n_pts/K < 0");
    if (!g->F64) return fail(FC_ERR_STATE, "fc_generate_universes: covariance not built");
    if (!g->lf_ok)
        return fail(FC_ERR_NOT_PD, "fc_generate_universes: fractional covariance not positive "
                                   "definite");
    if (K == 0) return FC_OK;
    if (n_pts < 1 || !p || !seg_off || !d)
        return fail(FC_ERR_INVALID_ARG, "fc_generate_universes: NULL device pointer or no points");
    hipError_t e = fcx::launch_gen_universes(g, n_pts, p, seg_off, u_first, seed, K, d, p_idx,
                                             counts, stream);
    if (e != hipSuccess) return hip_fail(e, "fc_generate_universes");
    return FC_OK;
}

int fc_region(const fc_grid *g, int32_t form, int64_t n_pts, const int64_t *pts, int64_t K0,
              int64_t K_max, double z, uint64_t seed, int32_t n_alpha, const double *alpha,
              const double *dchi2_data, double *crit, uint8_t *accepted, int64_t *K_used,
              int32_t *n_rounds, double *n_evals, hipStream_t stream)
{
    g_last_error.clear();
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_region: grid is NULL");
    if (form != FC_FORM_FP64 && form != FC_FORM_FP32 && form != FC_FORM_SPLIT_BF16 &&
        form != FC_FORM_SPLIT_FP16)
        return fail(FC_ERR_INVALID_ARG, "fc_region: bad form %d", form);
    if (!(g->forms & (uint32_t)form))
        return fail(FC_ERR_STATE, "fc_region: form %d was not built for this grid", form);
    if (!g->lf_ok)
        return fail(FC_ERR_NOT_PD, "fc_region: fractional covariance not positive definite");
    if (pts ? n_pts < 1 : n_pts != g->G)
        return fail(FC_ERR_INVALID_ARG, "fc_region: n_pts must be >= 1 (or G with pts NULL)");
    if (pts)
        for (int64_t k = 0; k < n_pts; ++k)
            if (pts[k] < 0 || pts[k] >= g->G)
                return fail(FC_ERR_INVALID_ARG, "fc_region: pts[%lld] outside the grid",
                            (long long)k);
    if (K0 < 1 || K_max < K0 || K_max > (int64_t(1) << 24))
        return fail(FC_ERR_INVALID_ARG, "fc_region: need 1 <= K0 <= K_max <= 2^24");
    if (!(z >= 0.0) || !std::isfinite(z)) return fail(FC_ERR_INVALID_ARG, "fc_region: bad z");
    if (n_alpha < 1 || n_alpha > 4 || !alpha)
        return fail(FC_ERR_INVALID_ARG, "fc_region: n_alpha must be 1..4");
    for (int a = 0; a < n_alpha; ++a)
        if (!(alpha[a] > 0.0 && alpha[a] <= 1.0))
            return fail(FC_ERR_INVALID_ARG, "fc_region: alpha[%d] not in (0,1]", a);
    if (!dchi2_data || !crit || !accepted || !K_used || !n_rounds || !n_evals)
        return fail(FC_ERR_INVALID_ARG, "fc_region: NULL argument");
    hipError_t e = hipSuccess;
    const int rc = fcx::region_run(g, form, n_pts, pts, K0, K_max, z, seed, n_alpha, alpha,
                                   dchi2_data, crit, accepted, K_used, n_rounds, n_evals, stream,
                                   &e);
    if (rc != FC_OK) {
        if (rc == FC_ERR_NOMEM) {
            (void)hipGetLastError();
            return fail(FC_ERR_NOMEM, "fc_region: device allocation failed (%s)",
                        hipGetErrorString(e));
        }
        return hip_fail(e, "fc_region");
    }
    return FC_OK;
}

int fc_scan_fixed_m(const fc_grid *g, int64_t K, const double *d, const int64_t *p_idx,
                    int32_t max_iter, double *dchi2, double *chi2_min, int64_t *argmin,
                    double *chi2_p, int64_t *m_final, int32_t *iters, hipStream_t stream)
{
    g_last_error.clear();
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_scan_fixed_m: grid is NULL");
    if (!(g->forms & FC_FORM_FP64))
        return fail(FC_ERR_STATE, "fc_scan_fixed_m: needs the FP64 form");
    if (K < 0 || K > (int64_t(1) << 30))
        return fail(FC_ERR_INVALID_ARG, "fc_scan_fixed_m: K=%lld not in 0..2^30", (long long)K);
    if (max_iter < 0 || max_iter > 64)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_fixed_m: max_iter=%d not in 0..64", max_iter);
    if (K == 0) return FC_OK;
    if (!d || !p_idx || !dchi2 || !chi2_min || !argmin || !chi2_p)
        return fail(FC_ERR_INVALID_ARG, "fc_scan_fixed_m: NULL device pointer");
    // true points are read back for the grouping: check them there
    std::vector<int64_t> hp(K);
    hipError_t e;
    if ((e = hipMemcpyAsync(hp.data(), p_idx, sizeof(int64_t) * K, hipMemcpyDeviceToHost,
                            stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return hip_fail(e, "fc_scan_fixed_m: read p_idx");
    for (int64_t k = 0; k < K; ++k)
        if (hp[k] < 0 || hp[k] >= g->G)
            return fail(FC_ERR_INVALID_ARG, "fc_scan_fixed_m: p_idx[%lld]=%lld outside the grid",
                        (long long)k, (long long)hp[k]);
    if ((e = fcx::fixed_run(g, K, d, p_idx, max_iter, dchi2, chi2_min, argmin, chi2_p, m_final,
                            iters, stream)) != hipSuccess)
        return hip_fail(e, "fc_scan_fixed_m");
    return FC_OK;
}

int fc_grid_inverse_cov(const fc_grid *g, int64_t q0, int64_t nq, double *out, hipStream_t stream)
{
    g_last_error.clear();
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_grid_inverse_cov: grid is NULL");
    if (!(g->forms & FC_FORM_FP64))
        return fail(FC_ERR_STATE, "fc_grid_inverse_cov: FP64 form not built");
    if (q0 < 0 || nq < 0 || q0 + nq > g->G)
        return fail(FC_ERR_INVALID_ARG, "fc_grid_inverse_cov: range out of the grid");
    if (nq == 0) return FC_OK;
    if (!out) return fail(FC_ERR_INVALID_ARG, "fc_grid_inverse_cov: out is NULL");
    if (nq > 0x7fffffff) return fail(FC_ERR_INVALID_ARG, "fc_grid_inverse_cov: nq too large");
    hipError_t e = fcx::launch_inverse_cov(g, q0, nq, out, stream);
    if (e != hipSuccess) return hip_fail(e, "fc_grid_inverse_cov: launch");
    return FC_OK;
}

int fc_grid_info(const fc_grid *g, int32_t *D, int32_t *N, int64_t *G, uint32_t *forms)
{
    g_last_error.clear();
    if (!g) return fail(FC_ERR_INVALID_ARG, "fc_grid_info: grid is NULL");
    if (D) *D = g->D;
    if (N) *N = g->N;
    if (G) *G = g->G;
    if (forms) *forms = g->forms;
    return FC_OK;
}

size_t fc_grid_device_bytes(const fc_grid *g) { return g ? g->bytes : 0; }

void fc_grid_destroy(fc_grid *g)
{
    if (!g) return;
    (void)hipDeviceSynchronize();
    free_forms(g);
    if (g->S64) (void)hipFree(g->S64);
    if (g->off) (void)hipFree(g->off);
    if (g->dev) (void)hipFree(g->dev);
    delete g;
}

}  // extern "C"
