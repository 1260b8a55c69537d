// fc_server.hip -- FC request serving with continuous batching (host runtime).
//
// Requests (one true point of one resident grid, K universes) are admitted in
// arrival order while their device memory fits a fixed arena.  A scheduler
// thread keeps at most two batched launches in flight per bin-count class; each
// launch is a persistent-style kernel over a table of work items (a tile of
// universes x a range of grid points) drawn from every admitted request of that
// class, so requests that arrive while others run join the next launch and
// share the device with them.  The two launch slots of a class run on two
// streams, so the next launch's blocks take the CUs that the current one's
// last items leave idle; a request's results are finalised once every launch
// holding its items has ended.  The device work per
// (universe, grid point) is the same code as fc_scan, and the running minimum
// is merged with an order-independent atomicMin, so a request's results do
// not depend on the mix it ran in.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <stdarg.h>
#include <stdio.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fc_internal.h"

extern "C" const char *fc_last_error(void);

namespace fcx {
int set_last_error(int code, const char *msg);
}

namespace {

using Clock = std::chrono::steady_clock;
double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return fcx::set_last_error(code, buf);
}

constexpr int kMaxItems = 16384;   // items per batched launch
constexpr int64_t kMaxK = int64_t(1) << 20;
constexpr int64_t kQStep = 256;     // grid points per item

// First-fit allocator of offsets inside one fixed region.
class Arena {
public:
    void init(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    static size_t round(size_t n) { return (n + 255) & ~size_t(255); }
    bool alloc(size_t n, size_t *off)
    {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

struct Req {
    int64_t id = 0;
    int grid = 0, cls = 0;
    int64_t p = 0, K = 0;
    int state = FC_REQ_QUEUED;
    double t_submit = 0.0, t_done = 0.0;
    size_t host_off = 0, host_bytes = 0, dev_off = 0, dev_bytes = 0;
    // device block
    double *d = nullptr, *chi2p = nullptr, *dchi2 = nullptr, *crit = nullptr;
    unsigned long long *keys = nullptr;
    int64_t *argmin = nullptr, *hist = nullptr, *seg = nullptr;
    // pinned host block
    double *h_d = nullptr, *h_dchi2 = nullptr, *h_cmin = nullptr, *h_chi2p = nullptr,
           *h_crit = nullptr;
    int64_t *h_argmin = nullptr, *h_hist = nullptr, *h_seg = nullptr;
    int64_t q_next = 0;
    bool finishing = false;
    hipEvent_t ev_done = nullptr;
    // universes drawn on the device instead of uploaded
    bool drawn = false;
    uint64_t seed = 0;
    int64_t u_first = 0;
    int64_t *pu = nullptr, *h_pu = nullptr;  // {p, u_first}
};

struct Cls {
    int ns = 0, code = 0, N = 0;  // code: the split layout (split_code)
    hipStream_t lst[2] = {nullptr, nullptr};   // stream of each launch slot
    hipEvent_t ev_admit[2] = {nullptr, nullptr};  // after the latest admission on lst[k]
    bool admit_wait[2] = {false, false};  // slot k must wait for ev_admit[k ^ 1]
    fcx::ScanItem *d_items[2] = {nullptr, nullptr};
    fcx::ScanItem *h_items[2] = {nullptr, nullptr};
    int *d_counter[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool busy[2] = {false, false};
    int next_slot = 0;
    int slots = 512;
    int upi = 128;
    size_t rr = 0;                  // round-robin start in `active`
    std::vector<int64_t> active;    // admitted requests with grid points left or finishing
};

}  // namespace

struct fc_server {
    int device = 0;
    int form = 0;
    std::vector<const fc_grid *> grids;
    std::vector<int> grid_cls;
    std::vector<Cls> classes;
    int n_alpha = 0, n_bins = 0;
    double alpha[8] = {0};
    double hist_hi = 0.0;
    double launch_evals = 0.0;
    int policy = FC_SCHED_FAIR;
    // memory
    void *dev_base = nullptr;
    void *host_base = nullptr;
    Arena dev_arena, host_arena;
    // requests
    std::mutex mu;
    std::condition_variable cv;
    std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
    std::deque<int64_t> queue;
    int64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    // stats
    int64_t n_done = 0, n_launches = 0;
    double evals = 0.0;
    bool device_error = false;
    std::string error_msg;

    void run();
    bool retire();
    bool admit();
    bool launch(Cls &c);
    void request_pointers(Req &r);
};

namespace {

// Both blocks hold the same pieces, each rounded to 256 B by carve():
// universes, segment offsets, {p, u_first}, dchi2, chi2_min (keys), chi2_p,
// argmin, crit, hist.  A request whose universes are drawn on the device has
// no universes in its host block.
size_t block_bytes(const fc_server *s, int64_t K, int N, bool with_universes)
{
    const size_t k = (size_t)K;
    return (with_universes ? Arena::round(sizeof(double) * k * N) : 0) +
           2 * Arena::round(sizeof(int64_t) * 2) + 4 * Arena::round(sizeof(double) * k) +
           Arena::round(sizeof(double) * s->n_alpha) +
           Arena::round(sizeof(int64_t) * (s->n_bins + 1));
}
size_t host_block_bytes(const fc_server *s, int64_t K, int N, bool drawn)
{
    return block_bytes(s, K, N, !drawn);
}
size_t dev_block_bytes(const fc_server *s, int64_t K, int N) { return block_bytes(s, K, N, true); }

template <typename T>
T *carve(char *&cur, size_t count)
{
    T *p = reinterpret_cast<T *>(cur);
    cur += Arena::round(sizeof(T) * count);
    return p;
}

}  // namespace

void fc_server::request_pointers(Req &r)
{
    const int N = grids[r.grid]->N;
    char *h = static_cast<char *>(host_base) + r.host_off;
    r.h_d = r.drawn ? nullptr : carve<double>(h, (size_t)r.K * N);
    r.h_seg = carve<int64_t>(h, 2);
    r.h_pu = carve<int64_t>(h, 2);
    r.h_dchi2 = carve<double>(h, r.K);
    r.h_cmin = carve<double>(h, r.K);
    r.h_chi2p = carve<double>(h, r.K);
    r.h_argmin = carve<int64_t>(h, r.K);
    r.h_crit = carve<double>(h, n_alpha);
    r.h_hist = carve<int64_t>(h, n_bins + 1);
}

bool fc_server::admit()
{
    bool progress = false;
    std::lock_guard<std::mutex> lk(mu);
    while (!queue.empty()) {
        Req &r = *reqs.at(queue.front());
        const int N = grids[r.grid]->N;
        r.dev_bytes = dev_block_bytes(this, r.K, N);
        if (!dev_arena.alloc(r.dev_bytes, &r.dev_off)) break;  // arrival order: wait for memory
        char *dv = static_cast<char *>(dev_base) + r.dev_off;
        r.d = carve<double>(dv, (size_t)r.K * N);
        r.keys = carve<unsigned long long>(dv, r.K);
        r.chi2p = carve<double>(dv, r.K);
        r.dchi2 = carve<double>(dv, r.K);
        r.argmin = carve<int64_t>(dv, r.K);
        r.crit = carve<double>(dv, n_alpha);
        r.hist = carve<int64_t>(dv, n_bins + 1);
        r.seg = carve<int64_t>(dv, 2);
        r.pu = carve<int64_t>(dv, 2);
        Cls &c = classes[r.cls];
        // admitted on the stream of the slot that launches next; the other
        // slot waits for it before its next launch
        const int a = c.next_slot;
        hipStream_t ast = c.lst[a];
        hipError_t e;
        if ((e = hipMemcpyAsync(r.seg, r.h_seg, sizeof(int64_t) * 2, hipMemcpyHostToDevice,
                                ast)) != hipSuccess ||
            (e = hipMemcpyAsync(r.pu, r.h_pu, sizeof(int64_t) * 2, hipMemcpyHostToDevice,
                                ast)) != hipSuccess ||
            (e = r.drawn ? fcx::launch_gen_universes(grids[r.grid], 1, r.pu, r.seg, r.pu + 1,
                                                     r.seed, r.K, r.d, nullptr, nullptr, ast)
                         : hipMemcpyAsync(r.d, r.h_d, sizeof(double) * (size_t)r.K * N,
                                          hipMemcpyHostToDevice, ast)) != hipSuccess ||
            (e = fcx::launch_init_keys(r.K, r.keys, r.chi2p, ast)) != hipSuccess ||
            (e = hipEventRecord(c.ev_admit[a], ast)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&r.ev_done, hipEventDisableTiming)) != hipSuccess) {
            device_error = true;
            error_msg = std::string("fc_server: admission: ") + hipGetErrorString(e);
            r.state = FC_REQ_FAILED;
            queue.pop_front();
            continue;
        }
        r.state = FC_REQ_RUNNING;
        r.q_next = 0;
        c.admit_wait[a ^ 1] = true;
        c.active.push_back(r.id);
        queue.pop_front();
        progress = true;
    }
    return progress;
}

bool fc_server::launch(Cls &c)
{
    int slot = -1;
    for (int k = 0; k < 2; ++k)
        if (!c.busy[(c.next_slot + k) & 1]) {
            slot = (c.next_slot + k) & 1;
            break;
        }
    if (slot < 0) return false;

    std::vector<Req *> order;
    {
        std::lock_guard<std::mutex> lk(mu);
        const size_t na = c.active.size();
        const size_t start = (policy == FC_SCHED_FAIR) ? c.rr : 0;  // FIFO: oldest first
        for (size_t k = 0; k < na; ++k) {
            Req *r = reqs.at(c.active[(start + k) % na]).get();
            if (r->state == FC_REQ_RUNNING && !r->finishing) order.push_back(r);
        }
        if (na) c.rr = (c.rr + 1) % na;
    }
    if (order.empty()) return false;

    fcx::ScanItem *items = c.h_items[slot];
    int n = 0;
    double budget = launch_evals, scheduled = 0.0;
    std::vector<Req *> completing;
    // FAIR: one range of grid points per request per round; FIFO: a request
    // takes ranges until it is fully scheduled before the next one is served
    bool any = true;
    while (any && budget > 0.0 && n < kMaxItems) {
        any = false;
        for (size_t oi = 0; oi < order.size(); ++oi) {
            Req *r = order[oi];
            const fc_grid *g = grids[r->grid];
            if (r->q_next >= g->G) continue;
            const int64_t ntiles = (r->K + c.upi - 1) / c.upi;
            if (n + ntiles > kMaxItems) continue;
            const int64_t qb = r->q_next;
            const int64_t qe = (qb + kQStep < g->G) ? qb + kQStep : g->G;
            for (int64_t t = 0; t < ntiles; ++t) {
                fcx::ScanItem &it = items[n++];
                it.R = (form == FC_FORM_FP32) ? g->R32 : (form == FC_FORM_SPLIT_FP16 ? g->RH16 : g->RB16);
                it.d = r->d;
                it.p_idx = nullptr;
                it.p = r->p;
                it.keys = r->keys;
                it.chi2_p = r->chi2p;
                it.off = g->off;
                it.K = r->K;
                it.u0 = t * c.upi;
                it.qb = qb;
                it.qe = qe;
                it.N = g->N;
                it.ed = (form == FC_FORM_SPLIT_FP16) ? g->ed16 : 0;
            }
            const double w = (double)r->K * (double)(qe - qb);
            budget -= w;
            scheduled += w;
            r->q_next = qe;
            any = true;
            if (r->q_next >= g->G) completing.push_back(r);
            if (budget <= 0.0 || n >= kMaxItems) break;
            if (policy == FC_SCHED_FIFO && r->q_next < g->G) --oi;  // stay on this request
        }
    }
    if (n == 0) return false;

    hipError_t e;
    const int blocks = n < c.slots ? n : c.slots;
    hipStream_t st = c.lst[slot];
    // admissions made on the other slot's stream (universes uploaded or drawn,
    // keys initialised) come first
    if (c.admit_wait[slot]) {
        if ((e = hipStreamWaitEvent(st, c.ev_admit[slot ^ 1], 0)) != hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            device_error = true;
            error_msg = std::string("fc_server: wait: ") + hipGetErrorString(e);
            return false;
        }
        c.admit_wait[slot] = false;
    }
    if ((e = hipMemcpyAsync(c.d_items[slot], items, sizeof(fcx::ScanItem) * n,
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemsetAsync(c.d_counter[slot], 0, sizeof(int), st)) != hipSuccess ||
        (e = (form == FC_FORM_FP32)
                 ? fcx::launch_serve_fp32(c.N, c.d_items[slot], n, c.d_counter[slot], blocks, st)
                 : fcx::launch_serve_split(c.code, form == FC_FORM_SPLIT_FP16,
                                           c.d_items[slot], n, c.d_counter[slot], blocks,
                                           st)) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        device_error = true;
        error_msg = std::string("fc_server: launch: ") + hipGetErrorString(e);
        return false;
    }
    // requests whose last items are in this launch: finalize, critical values,
    // copy back.  Their earlier items are in earlier launches of this stream
    // (stream order) or in the other slot's launches: wait for the latest of
    // those if it may still run.
    const int other = slot ^ 1;
    if (!completing.empty() && c.busy[other] &&
        (e = hipStreamWaitEvent(st, c.ev[other], 0)) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        device_error = true;
        error_msg = std::string("fc_server: wait: ") + hipGetErrorString(e);
        return false;
    }
    for (Req *r : completing) {
        const size_t K = (size_t)r->K;
        if ((e = fcx::launch_finalize(r->K, nullptr, r->keys, reinterpret_cast<double *>(r->keys),
                                      r->argmin, r->chi2p, r->dchi2, st, r->p)) !=
                hipSuccess ||
            (e = fcx::launch_crit(1, r->seg, r->dchi2, n_alpha, alpha, r->crit, n_bins, hist_hi,
                                  r->hist, st)) != hipSuccess ||
            (e = hipMemcpyAsync(r->h_dchi2, r->dchi2, sizeof(double) * K, hipMemcpyDeviceToHost,
                                st)) != hipSuccess ||
            (e = hipMemcpyAsync(r->h_cmin, r->keys, sizeof(double) * K, hipMemcpyDeviceToHost,
                                st)) != hipSuccess ||
            (e = hipMemcpyAsync(r->h_chi2p, r->chi2p, sizeof(double) * K, hipMemcpyDeviceToHost,
                                st)) != hipSuccess ||
            (e = hipMemcpyAsync(r->h_argmin, r->argmin, sizeof(int64_t) * K,
                                hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipMemcpyAsync(r->h_crit, r->crit, sizeof(double) * n_alpha,
                                hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipMemcpyAsync(r->h_hist, r->hist, sizeof(int64_t) * (n_bins + 1),
                                hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipEventRecord(r->ev_done, st)) != hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            device_error = true;
            error_msg = std::string("fc_server: finish: ") + hipGetErrorString(e);
            return false;
        }
        r->finishing = true;
    }
    if ((e = hipEventRecord(c.ev[slot], st)) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        device_error = true;
        error_msg = std::string("fc_server: event: ") + hipGetErrorString(e);
        return false;
    }
    c.busy[slot] = true;
    c.next_slot = slot ^ 1;
    std::lock_guard<std::mutex> lk(mu);
    n_launches += 1;
    evals += scheduled;
    return true;
}

bool fc_server::retire()
{
    bool progress = false;
    for (Cls &c : classes)
        for (int k = 0; k < 2; ++k)
            if (c.busy[k]) {
                const hipError_t e = hipEventQuery(c.ev[k]);
                if (e == hipSuccess) {
                    c.busy[k] = false;
                    progress = true;
                } else if (e != hipErrorNotReady) {
                    std::lock_guard<std::mutex> lk(mu);
                    device_error = true;
                    error_msg = std::string("fc_server: launch failed: ") + hipGetErrorString(e);
                    c.busy[k] = false;
                }
            }
    std::lock_guard<std::mutex> lk(mu);
    for (Cls &c : classes) {
        for (size_t k = 0; k < c.active.size();) {
            Req &r = *reqs.at(c.active[k]);
            if (r.finishing) {
                const hipError_t e = hipEventQuery(r.ev_done);
                if (e != hipErrorNotReady) {
                    r.t_done = now_s();
                    r.state = (e == hipSuccess) ? FC_REQ_DONE : FC_REQ_FAILED;
                    (void)hipEventDestroy(r.ev_done);
                    r.ev_done = nullptr;
                    dev_arena.release(r.dev_off, r.dev_bytes);
                    r.finishing = false;
                    c.active.erase(c.active.begin() + (long)k);
                    if (c.rr >= c.active.size()) c.rr = 0;
                    n_done += 1;
                    progress = true;
                    cv.notify_all();
                    continue;
                }
            }
            ++k;
        }
    }
    return progress;
}

void fc_server::run()
{
    (void)hipSetDevice(device);
    for (;;) {
        bool progress = retire();
        {
            // a device error ends every request that is not done
            std::lock_guard<std::mutex> lk(mu);
            if (device_error) {
                for (auto &kv : reqs)
                    if (kv.second->state == FC_REQ_QUEUED || kv.second->state == FC_REQ_RUNNING)
                        kv.second->state = FC_REQ_FAILED;
                queue.clear();
                for (Cls &c : classes) c.active.clear();
                stop = true;
                cv.notify_all();
            }
        }
        bool stopping, in_flight = false;
        {
            std::lock_guard<std::mutex> lk(mu);
            stopping = stop;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Cls &c : classes) {
                in_flight = in_flight || c.busy[0] || c.busy[1];
                for (int64_t id : c.active)
                    if (reqs.at(id)->finishing) in_flight = true;
            }
        }
        if (stopping && !in_flight) break;
        if (!stopping) {
            progress = admit() || progress;
            for (Cls &c : classes) progress = launch(c) || progress;
        }
        if (!progress) {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait_for(lk, std::chrono::microseconds(50));
        }
    }
}

extern "C" {

int fc_server_create(fc_server **out, const fc_grid *const *grids, int32_t n_grids, int32_t form,
                     size_t hbm_budget, size_t host_budget, int32_t n_alpha, const double *alpha,
                     int32_t n_bins, double hist_hi, double launch_evals, int32_t policy)
{
    if (!out) return fail(FC_ERR_INVALID_ARG, "fc_server_create: out is NULL");
    *out = nullptr;
    if (!grids || n_grids < 1 || n_grids > 64)
        return fail(FC_ERR_INVALID_ARG, "fc_server_create: need 1..64 grids");
    if (form != FC_FORM_FP32 && form != FC_FORM_SPLIT_BF16 && form != FC_FORM_SPLIT_FP16)
        return fail(FC_ERR_INVALID_ARG, "fc_server_create: form must be FP32 or a split form");
    if (n_alpha < 1 || n_alpha > 8 || !alpha)
        return fail(FC_ERR_INVALID_ARG, "fc_server_create: n_alpha must be 1..8");
    for (int a = 0; a < n_alpha; ++a)
        if (!(alpha[a] > 0.0 && alpha[a] <= 1.0))
            return fail(FC_ERR_INVALID_ARG, "fc_server_create: alpha[%d] not in (0,1]", a);
    if (n_bins < 1 || n_bins > 16383 || !(hist_hi > 0.0) || !std::isfinite(hist_hi))
        return fail(FC_ERR_INVALID_ARG, "fc_server_create: bad histogram settings");
    if (hbm_budget < (size_t(1) << 20) || host_budget < (size_t(1) << 20))
        return fail(FC_ERR_INVALID_ARG, "fc_server_create: budgets must be >= 1 MiB");
    if (!(launch_evals >= 0.0)) return fail(FC_ERR_INVALID_ARG, "fc_server_create: launch_evals");
    if (policy != FC_SCHED_FAIR && policy != FC_SCHED_FIFO)
        return fail(FC_ERR_INVALID_ARG, "fc_server_create: bad policy %d", policy);
    for (int i = 0; i < n_grids; ++i) {
        if (!grids[i]) return fail(FC_ERR_INVALID_ARG, "fc_server_create: grid %d is NULL", i);
        if (!(grids[i]->forms & (uint32_t)form))
            return fail(FC_ERR_STATE, "fc_server_create: grid %d lacks the form", i);
    }
    std::unique_ptr<fc_server> s(new (std::nothrow) fc_server());
    if (!s) return fail(FC_ERR_NOMEM, "fc_server_create: host allocation");
    (void)hipGetDevice(&s->device);
    s->form = form;
    s->n_alpha = n_alpha;
    for (int a = 0; a < n_alpha; ++a) s->alpha[a] = alpha[a];
    s->n_bins = n_bins;
    s->hist_hi = hist_hi;
    s->launch_evals = launch_evals > 0.0 ? launch_evals : (form == FC_FORM_FP32 ? 1.5e8 : 4.5e8);
    s->policy = policy;
    s->grids.assign(grids, grids + n_grids);
    // one class per distinct kernel geometry
    for (int i = 0; i < n_grids; ++i) {
        const int N = grids[i]->N;
        int found = -1;
        for (size_t c = 0; c < s->classes.size(); ++c) {
            const Cls &cl = s->classes[c];
            const bool same = (form == FC_FORM_FP32)
                                  ? cl.N == N
                                  : cl.code == fcx::split_code(N);
            if (same) found = (int)c;
        }
        if (found < 0) {
            Cls cl;
            cl.N = N;
            cl.ns = fcx::n_ksteps(N);
            cl.code = fcx::split_code(N);
            s->classes.push_back(cl);
            found = (int)s->classes.size() - 1;
        }
        s->grid_cls.push_back(found);
    }
    hipError_t e;
    auto cleanup_fail = [&](const char *what) {
        for (Cls &c : s->classes) {
            for (int k = 0; k < 2; ++k) {
                if (c.d_items[k]) (void)hipFree(c.d_items[k]);
                if (c.h_items[k]) (void)hipHostFree(c.h_items[k]);
                if (c.d_counter[k]) (void)hipFree(c.d_counter[k]);
                if (c.ev[k]) (void)hipEventDestroy(c.ev[k]);
                if (c.ev_admit[k]) (void)hipEventDestroy(c.ev_admit[k]);
                if (c.lst[k]) (void)hipStreamDestroy(c.lst[k]);
            }
        }
        if (s->dev_base) (void)hipFree(s->dev_base);
        if (s->host_base) (void)hipHostFree(s->host_base);
        return fail(e == hipErrorOutOfMemory ? FC_ERR_NOMEM : FC_ERR_DEVICE, "%s: %s", what,
                    hipGetErrorString(e));
    };
    if ((e = hipMalloc(&s->dev_base, hbm_budget)) != hipSuccess)
        return cleanup_fail("fc_server_create: device budget");
    if ((e = hipHostMalloc(&s->host_base, host_budget, hipHostMallocDefault)) != hipSuccess)
        return cleanup_fail("fc_server_create: host budget");
    s->dev_arena.init(hbm_budget);
    s->host_arena.init(host_budget);
    for (Cls &c : s->classes) {
        for (int k = 0; k < 2; ++k)
            if ((e = hipStreamCreateWithFlags(&c.lst[k], hipStreamNonBlocking)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&c.ev_admit[k], hipEventDisableTiming)) !=
                    hipSuccess)
                return cleanup_fail("fc_server_create: stream");
        for (int k = 0; k < 2; ++k) {
            if ((e = hipMalloc(&c.d_items[k], sizeof(fcx::ScanItem) * kMaxItems)) != hipSuccess ||
                (e = hipHostMalloc(reinterpret_cast<void **>(&c.h_items[k]),
                                   sizeof(fcx::ScanItem) * kMaxItems, hipHostMallocDefault)) !=
                    hipSuccess ||
                (e = hipMalloc(&c.d_counter[k], sizeof(int))) != hipSuccess ||
                (e = hipEventCreateWithFlags(&c.ev[k], hipEventDisableTiming)) != hipSuccess)
                return cleanup_fail("fc_server_create: launch tables");
        }
        if (s->form == FC_FORM_FP32) {
            c.slots = fcx::serve_slots_fp32(c.N);
            c.upi = fcx::serve_fp32_univ_per_item();
        } else {
            c.slots = fcx::serve_slots_split(c.code, s->form == FC_FORM_SPLIT_FP16);
            c.upi = fcx::serve_split_univ_per_item();
        }
    }
    fc_server *raw = s.release();
    raw->worker = std::thread([raw] { raw->run(); });
    *out = raw;
    return FC_OK;
}

namespace {

int submit_common(fc_server *s, int32_t grid, int64_t p, int64_t K, const double *d, bool drawn,
                  uint64_t seed, int64_t u_first, int64_t *req, const char *who)
{
    if (!s || !req) return fail(FC_ERR_INVALID_ARG, "%s: NULL argument", who);
    if (grid < 0 || grid >= (int32_t)s->grids.size())
        return fail(FC_ERR_INVALID_ARG, "%s: grid %d out of range", who, grid);
    const fc_grid *g = s->grids[grid];
    if (p < 0 || p >= g->G)
        return fail(FC_ERR_INVALID_ARG, "%s: p=%lld out of range", who, (long long)p);
    if (K < 1 || K > kMaxK)
        return fail(FC_ERR_INVALID_ARG, "%s: K=%lld not in 1..2^20", who, (long long)K);
    if (!drawn && !d) return fail(FC_ERR_INVALID_ARG, "%s: d is NULL", who);
    if (drawn && u_first < 0) return fail(FC_ERR_INVALID_ARG, "%s: u_first < 0", who);
    if (drawn && !g->lf_ok)
        return fail(FC_ERR_NOT_PD, "%s: the grid's fractional covariance has no factor", who);
    const size_t dev = Arena::round(dev_block_bytes(s, K, g->N));
    if (dev > s->dev_arena.size())
        return fail(FC_ERR_NOMEM, "%s: request needs %zu B > device budget %zu B", who, dev,
                    s->dev_arena.size());
    std::unique_ptr<Req> r(new (std::nothrow) Req());
    if (!r) return fail(FC_ERR_NOMEM, "%s: host allocation", who);
    r->grid = grid;
    r->cls = s->grid_cls[grid];
    r->p = p;
    r->K = K;
    r->drawn = drawn;
    r->seed = seed;
    r->u_first = u_first;
    r->host_bytes = host_block_bytes(s, K, g->N, drawn);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->device_error) return fail(FC_ERR_DEVICE, "%s", s->error_msg.c_str());
        if (!s->host_arena.alloc(r->host_bytes, &r->host_off))
            return fail(FC_ERR_NOMEM, "%s: host staging memory exhausted", who);
    }
    s->request_pointers(*r);
    if (!drawn) std::memcpy(r->h_d, d, sizeof(double) * (size_t)K * g->N);
    r->h_seg[0] = 0;
    r->h_seg[1] = K;
    r->h_pu[0] = p;
    r->h_pu[1] = u_first;
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    *req = r->id;
    s->queue.push_back(r->id);
    s->reqs.emplace(r->id, std::move(r));
    s->cv.notify_all();
    return FC_OK;
}

}  // namespace

int fc_server_submit(fc_server *s, int32_t grid, int64_t p, int64_t K, const double *d,
                     int64_t *req)
{
    return submit_common(s, grid, p, K, d, false, 0, 0, req, "fc_server_submit");
}

int fc_server_submit_drawn(fc_server *s, int32_t grid, int64_t p, int64_t K, uint64_t seed,
                           int64_t u_first, int64_t *req)
{
    return submit_common(s, grid, p, K, nullptr, true, seed, u_first, req,
                         "fc_server_submit_drawn");
}

int fc_server_poll(fc_server *s, int64_t req, int32_t *state, double *dchi2, double *chi2_min,
                   int64_t *argmin, double *chi2_p, double *crit, int64_t *hist, double *latency,
                   int32_t release)
{
    if (!s || !state) return fail(FC_ERR_INVALID_ARG, "fc_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req);
    if (it == s->reqs.end())
        return fail(FC_ERR_INVALID_ARG, "fc_server_poll: unknown request %lld", (long long)req);
    Req &r = *it->second;
    *state = r.state;
    if (r.state == FC_REQ_FAILED)
        return fail(FC_ERR_DEVICE, "fc_server_poll: request failed: %s", s->error_msg.c_str());
    if (r.state != FC_REQ_DONE) return FC_OK;
    const size_t K = (size_t)r.K;
    if (dchi2) std::memcpy(dchi2, r.h_dchi2, sizeof(double) * K);
    if (chi2_min) std::memcpy(chi2_min, r.h_cmin, sizeof(double) * K);
    if (argmin) std::memcpy(argmin, r.h_argmin, sizeof(int64_t) * K);
    if (chi2_p) std::memcpy(chi2_p, r.h_chi2p, sizeof(double) * K);
    if (crit) std::memcpy(crit, r.h_crit, sizeof(double) * s->n_alpha);
    if (hist) std::memcpy(hist, r.h_hist, sizeof(int64_t) * (s->n_bins + 1));
    if (latency) *latency = r.t_done - r.t_submit;
    if (release) {
        s->host_arena.release(r.host_off, r.host_bytes);
        s->reqs.erase(it);
    }
    return FC_OK;
}

int fc_server_stats(fc_server *s, int64_t *done, int64_t *launches, double *evals,
                    size_t *hbm_in_use)
{
    if (!s) return fail(FC_ERR_INVALID_ARG, "fc_server_stats: server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (done) *done = s->n_done;
    if (launches) *launches = s->n_launches;
    if (evals) *evals = s->evals;
    if (hbm_in_use) *hbm_in_use = s->dev_arena.used();
    return FC_OK;
}

void fc_server_destroy(fc_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (Cls &c : s->classes) {
        for (int k = 0; k < 2; ++k)
            if (c.lst[k]) (void)hipStreamSynchronize(c.lst[k]);
        for (int k = 0; k < 2; ++k) {
            if (c.d_items[k]) (void)hipFree(c.d_items[k]);
            if (c.h_items[k]) (void)hipHostFree(c.h_items[k]);
            if (c.d_counter[k]) (void)hipFree(c.d_counter[k]);
            if (c.ev[k]) (void)hipEventDestroy(c.ev[k]);
            if (c.ev_admit[k]) (void)hipEventDestroy(c.ev_admit[k]);
            if (c.lst[k]) (void)hipStreamDestroy(c.lst[k]);
        }
    }
    for (auto &kv : s->reqs)
        if (kv.second->ev_done) (void)hipEventDestroy(kv.second->ev_done);
    if (s->dev_base) (void)hipFree(s->dev_base);
    if (s->host_base) (void)hipHostFree(s->host_base);
    delete s;
}

}  // extern "C"
