// Continuous-batching server of polar requests (la_serve_* in la.h).
//
// One scheduler thread per server drives a HIP stream in "ticks".  A tick:
//   1. admits queued requests (FIFO) while a slot is free and the request's
//      device footprint fits the arena (first-fit allocator); for each, the
//      input is copied in and ||A||_F taken in FP64 (Algorithm NS_Polar,
//      first step), then X0 = A / ||A||_F;
//   2. advances every active request by one iteration of Algorithm NS_Polar
//      (a preconditioning step, eqs. a_def-RogueMatrix, or a Newton-Schulz
//      step, eq. NewtonSchulz): one grouped Gram launch and one grouped update
//      launch per precision cover all requests, whatever their sizes;
//   3. reduces the step norms of the Newton-Schulz requests in one grouped
//      launch and reads them back in one copy (the only per-tick sync);
//   4. applies each request's stop test on the host; finished requests get
//      H = sym(U^T A) in one grouped launch, their factors are copied to
//      pinned host buffers and their arena blocks are released.
// Every tile of every request is computed by the same kernel code with the
// same tile shape as when the request runs alone, so a request's result is
// bitwise independent of what else is in flight.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "la_internal.h"

namespace la {
namespace {

constexpr size_t kAlign = 256;
constexpr size_t kDescBytes = 1u << 20;      // GemmDesc arrays
constexpr size_t kItemBytes = 6u << 20;      // GroupItem arrays
constexpr size_t kRedBytes = 1u << 20;       // ReduceItem arrays + step norms
constexpr size_t kReserve = kDescBytes + kItemBytes + kRedBytes;

size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over [lo, hi) with coalescing of freed blocks.
class Arena {
  public:
    void init(size_t lo, size_t hi)
    {
        free_.clear();
        if (hi > lo)
            free_[lo] = hi - lo;
        used_ = 0;
        high_ = 0;
        cap_ = hi > lo ? hi - lo : 0;
    }
    size_t capacity() const { return cap_; }
    bool alloc(size_t size, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= size) {
                *off = it->first;
                const size_t rest = it->second - size;
                const size_t noff = it->first + size;
                free_.erase(it);
                if (rest)
                    free_[noff] = rest;
                used_ += size;
                high_ = std::max(high_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t size)
    {
        used_ -= size;
        auto it = free_.emplace(off, size).first;
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
    size_t high_water() const { return high_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, high_ = 0, cap_ = 0;
};

enum State { QUEUED, ACTIVE, DONE };

struct Req {
    uint64_t id;
    int64_t m, n;
    PolarPlan plan;
    State state = QUEUED;
    la_status status = LA_OK;
    // pinned host staging: the input A, reused for the result U (both m x n;
    // the upload has completed before U is copied back), and H
    float *io_pinned = nullptr;
    float *h_pinned = nullptr;
    // device state, carved from the arena block
    size_t off = 0, bytes = 0;
    float *A = nullptr, *X[2] = {nullptr, nullptr}, *P = nullptr;
    double *tiles = nullptr, *sumsq = nullptr, *scal = nullptr;
    int cur = 0;
    bool stopped = false;    // stop test passed (a polish step may follow)
    bool finished = false;   // no more iterations
    double prev_delta = INFINITY;
    la_polar_info info{};
    double t_submit = 0, t_done = 0;
};

// Most update tiles any precision uses for an m x n iterate.
size_t max_tiles(int64_t m, int64_t n)
{
    size_t t = 0;
    for (int pr : {PREC_FP32, PREC_BF16X3, PREC_BF16X6})
        t = std::max(t, (size_t)((m + tile_m(pr, 1) - 1) / tile_m(pr, 1)) *
                            (size_t)((n + tile_n(pr, 1) - 1) / tile_n(pr, 1)));
    return t;
}

// Bytes of one request's device state.
size_t footprint(int64_t m, int64_t n)
{
    const size_t mn = (size_t)m * n, nn = (size_t)n * n;
    return up(mn * 4) * 3 + up(nn * 4) + up(max_tiles(m, n) * 8) +
           up((size_t)sumsq_num_partials() * 8) + up(8 * 8);
}

}  // namespace
}  // namespace la

using namespace la;

struct la_server {
    la_context *ctx = nullptr;
    int device = 0;
    int max_slots = 32, max_queue = 4096;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    Arena alloc;
    hipStream_t stream = nullptr;
    // pinned host staging (descriptors, items, step norms)
    char *h_stage = nullptr;
    double *h_deltas = nullptr;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> all;
    uint64_t next_id = 1;
    bool stop = false;
    la_serve_stats stats{};
    std::thread worker;
    la_status fatal = LA_OK;

    void run();
    void tick();
    void fail(Req *r, la_status st)
    {
        r->status = st;
        r->finished = true;
    }
};

namespace {

// Carve a request's block.
void carve(Req *r, char *base)
{
    char *b = base + r->off;
    const size_t mn = (size_t)r->m * r->n, nn = (size_t)r->n * r->n;
    r->A = (float *)b;
    b += up(mn * 4);
    r->X[0] = (float *)b;
    b += up(mn * 4);
    r->X[1] = (float *)b;
    b += up(mn * 4);
    r->P = (float *)b;
    b += up(nn * 4);
    r->tiles = (double *)b;
    b += up(max_tiles(r->m, r->n) * 8);
    r->sumsq = (double *)b;
    b += up((size_t)sumsq_num_partials() * 8);
    r->scal = (double *)b;
}

struct Launch {
    int prec, akc, bkc, small;
    std::vector<GemmDesc> probs;
    std::vector<GroupItem> items;
};

}  // namespace

// Upload descriptors and items of each launch to the arena's reserved area
// and run the grouped kernels; items are ordered by decreasing K so the
// persistent workgroups share the work evenly.
static hipError_t run_launches(la_server *s, std::vector<Launch> &ls, size_t &dpos, size_t &ipos)
{
    for (auto &L : ls) {
        if (L.items.empty())
            continue;
        std::stable_sort(L.items.begin(), L.items.end(), [&](const GroupItem &x, const GroupItem &y) {
            return L.probs[x.prob].K > L.probs[y.prob].K;
        });
        const size_t db = L.probs.size() * sizeof(GemmDesc);
        const size_t ib = L.items.size() * sizeof(GroupItem);
        if (dpos + db > kDescBytes || ipos + ib > kItemBytes)
            return hipErrorOutOfMemory;
        memcpy(s->h_stage + dpos, L.probs.data(), db);
        memcpy(s->h_stage + kDescBytes + ipos, L.items.data(), ib);
        GemmDesc *dd = (GemmDesc *)(s->arena + dpos);
        GroupItem *di = (GroupItem *)(s->arena + kDescBytes + ipos);
        hipError_t e = hipMemcpyAsync(dd, s->h_stage + dpos, db, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(di, s->h_stage + kDescBytes + ipos, ib, hipMemcpyHostToDevice,
                               s->stream);
        if (e == hipSuccess)
            e = launch_gemm_grouped(L.prec, L.akc, L.bkc, L.small, dd, di, (int)L.items.size(),
                                    s->ctx->num_cus, s->stream);
        if (e != hipSuccess)
            return e;
        dpos += up(db);
        ipos += up(ib);
    }
    return hipSuccess;
}

static void add_problem(std::vector<Launch> &ls, int prec, int akc, int bkc, const GemmDesc &d)
{
    Launch *L = nullptr;
    for (auto &x : ls)
        if (x.prec == prec && x.akc == akc && x.bkc == bkc && x.small == d.small)
            L = &x;
    if (!L) {
        ls.push_back(Launch{prec, akc, bkc, d.small, {}, {}});
        L = &ls.back();
    }
    const int pid = (int)L->probs.size();
    L->probs.push_back(d);
    for (int t = 0; t < d.num_tiles; ++t)
        L->items.push_back(GroupItem{pid, t});
}

void la_server::tick()
{
    const double t0 = now_s();
    std::vector<Req *> fresh;
    {
        std::lock_guard<std::mutex> g(mu);
        while (!queue.empty() && (int)active.size() < max_slots) {
            Req *r = queue.front();
            size_t off;
            if (!alloc.alloc(r->bytes, &off))
                break;
            queue.pop_front();
            r->off = off;
            r->state = ACTIVE;
            carve(r, arena);
            active.push_back(r);
            fresh.push_back(r);
        }
        stats.queued = (int)queue.size();
        stats.active = (int)active.size();
        stats.arena_high_water = alloc.high_water() + kReserve;
    }
    hipError_t e = hipSuccess;
    // 1. newly admitted: upload, ||A||_F in FP64
    for (Req *r : fresh) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->A, r->io_pinned, (size_t)r->m * r->n * 4,
                               hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = launch_sumsq(r->A, r->m, r->n, r->n, r->sumsq, stream);
        if (e == hipSuccess)
            e = launch_reduce_fixed(r->sumsq, sumsq_num_partials(), r->scal, stream);
    }
    for (size_t i = 0; i < fresh.size() && e == hipSuccess; ++i)
        e = hipMemcpyAsync(h_deltas + i, fresh[i]->scal, 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess && !fresh.empty())
        e = hipStreamSynchronize(stream);
    for (size_t i = 0; i < fresh.size() && e == hipSuccess; ++i) {
        Req *r = fresh[i];
        const double fro = sqrt(h_deltas[i]);
        r->info.fro_norm_a = fro;
        if (!(fro > 0.0) || !isfinite(fro)) {
            fail(r, LA_ERR_NONFINITE);
            continue;
        }
        e = launch_scale(r->A, r->n, r->X[0], r->n, r->m, r->n, fro, stream);
        r->cur = 0;
    }
    // 2. one iteration for every running request
    std::vector<Req *> run;
    for (Req *r : active)
        if (!r->finished)
            run.push_back(r);
    std::vector<Launch> grams, updates;
    std::vector<Req *> ns;
    std::vector<int64_t> ntiles_ns;
    for (Req *r : run) {
        const PolarPlan &p = r->plan;
        const bool pre = r->info.iters_precond < p.k_pre;
        const int prec = pre ? p.prec_pre : (r->stopped ? PREC_BF16X6 : p.prec_ns);
        const int n = (int)r->n;
        GemmDesc gd;
        memset(&gd, 0, sizeof gd);
        gd.A = r->X[r->cur];
        gd.lda = n;
        gd.B = r->X[r->cur];
        gd.ldb = n;
        gd.C = r->P;
        gd.ldc = n;
        gd.M = n;
        gd.N = n;
        gd.K = r->m;
        gd.alpha = pre ? (float)(-p.c) : -1.0f;
        gd.gamma = 1.0f;
        gd.gram = 1;
        gemm_finalize(gd, prec);
        add_problem(grams, prec, 0, 0, gd);
        GemmDesc ud;
        memset(&ud, 0, sizeof ud);
        ud.A = r->X[r->cur];
        ud.lda = n;
        ud.a_kcontig = 1;
        ud.B = r->P;
        ud.ldb = n;
        ud.C = r->X[r->cur ^ 1];
        ud.ldc = n;
        ud.M = r->m;
        ud.N = n;
        ud.K = n;
        if (pre) {
            ud.alpha = (float)p.a;
        } else {
            ud.alpha = 0.5f;
            ud.beta = 1.0f;
            ud.E = r->X[r->cur];
            ud.lde = n;
            ud.partials = r->tiles;
            ns.push_back(r);
        }
        gemm_finalize(ud, prec);
        if (!pre)
            ntiles_ns.push_back((int64_t)ud.tiles_m * ud.tiles_n);
        add_problem(updates, prec, 1, 0, ud);
    }
    size_t dpos = 0, ipos = 0;  // staging offsets; reset only after a sync
    if (e == hipSuccess)
        e = run_launches(this, grams, dpos, ipos);
    if (e == hipSuccess)
        e = run_launches(this, updates, dpos, ipos);
    // 3. step norms of the Newton-Schulz requests
    if (e == hipSuccess && !ns.empty()) {
        std::vector<ReduceItem> ri(ns.size());
        double *dev_d = (double *)(arena + kDescBytes + kItemBytes);
        ReduceItem *dev_ri = (ReduceItem *)(arena + kDescBytes + kItemBytes + 4096 * 8);
        for (size_t i = 0; i < ns.size(); ++i)
            ri[i] = ReduceItem{ns[i]->tiles, ntiles_ns[i], dev_d + i};
        char *hst = h_stage + kDescBytes + kItemBytes;
        memcpy(hst, ri.data(), ri.size() * sizeof(ReduceItem));
        e = hipMemcpyAsync(dev_ri, hst, ri.size() * sizeof(ReduceItem), hipMemcpyHostToDevice,
                           stream);
        if (e == hipSuccess)
            e = launch_reduce_grouped(dev_ri, (int)ns.size(), stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_deltas, dev_d, ns.size() * 8, hipMemcpyDeviceToHost, stream);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        set_error("la_serve: device error %s", hipGetErrorString(e));
        std::lock_guard<std::mutex> g(mu);
        fatal = LA_ERR_DEVICE;
        for (Req *r : active)
            fail(r, LA_ERR_DEVICE);
    }
    // 4. host decisions (the stop test of Algorithm NS_Polar)
    if (e == hipSuccess) {
        size_t k = 0;
        for (Req *r : run) {
            const PolarPlan &p = r->plan;
            r->cur ^= 1;
            if (r->info.iters_precond < p.k_pre) {
                r->info.iters_precond++;
                continue;
            }
            const double delta = sqrt(h_deltas[k++]);
            r->info.iters_ns++;
            r->info.last_delta = delta;
            if (!isfinite(delta)) {
                fail(r, LA_ERR_NONFINITE);
                continue;
            }
            if (r->stopped) {  // polish step done
                r->finished = true;
                continue;
            }
            const double tol = (double)std::max(r->m, r->n) * p.eps;
            if (delta <= tol) {
                r->info.stop_reason = 0;
                r->stopped = true;
            } else if (p.stagnation && delta < 1e-2 * sqrt((double)r->n) &&
                       delta > 0.5 * r->prev_delta) {
                r->info.stop_reason = 1;
                r->stopped = true;
            }
            r->prev_delta = delta;
            if (r->stopped && !p.polish)
                r->finished = true;
            if (!r->stopped && r->info.iters_ns >= p.max_iter) {
                r->info.stop_reason = 2;
                r->status = LA_ERR_NOT_CONVERGED;
                r->finished = true;
            }
        }
    }
    // 5. finished requests: H, results to host, release
    std::vector<Req *> done;
    for (Req *r : active)
        if (r->finished)
            done.push_back(r);
    if (!done.empty()) {
        std::vector<Launch> hs;
        for (Req *r : done) {
            if (r->status != LA_OK && r->status != LA_ERR_NOT_CONVERGED)
                continue;
            GemmDesc hd;
            memset(&hd, 0, sizeof hd);
            hd.A = r->X[r->cur];
            hd.lda = r->n;
            hd.B = r->A;
            hd.ldb = r->n;
            hd.C = r->P;
            hd.ldc = r->n;
            hd.M = r->n;
            hd.N = r->n;
            hd.K = r->m;
            hd.alpha = 1.0f;
            gemm_finalize(hd, r->plan.prec_h);
            add_problem(hs, r->plan.prec_h, 0, 0, hd);
        }
        size_t dpos2 = 0, ipos2 = 0;  // the stream was synchronised above
        hipError_t e2 = e == hipSuccess ? run_launches(this, hs, dpos2, ipos2) : e;
        for (Req *r : done) {
            if (e2 != hipSuccess || (r->status != LA_OK && r->status != LA_ERR_NOT_CONVERGED))
                continue;
            e2 = launch_symmetrize(r->P, r->n, r->n, stream);
            if (e2 == hipSuccess)
                e2 = hipMemcpyAsync(r->io_pinned, r->X[r->cur], (size_t)r->m * r->n * 4,
                                    hipMemcpyDeviceToHost, stream);
            if (e2 == hipSuccess && r->h_pinned)
                e2 = hipMemcpyAsync(r->h_pinned, r->P, (size_t)r->n * r->n * 4,
                                    hipMemcpyDeviceToHost, stream);
        }
        if (e2 == hipSuccess)
            e2 = hipStreamSynchronize(stream);
        const double t1 = now_s();
        std::lock_guard<std::mutex> g(mu);
        for (Req *r : done) {
            if (e2 != hipSuccess && r->status == LA_OK)
                r->status = LA_ERR_DEVICE;
            r->state = DONE;
            r->t_done = t1;
            r->info.prec_precond = r->plan.prec_pre;
            r->info.prec_ns = r->plan.prec_ns;
            r->info.prec_h = r->plan.prec_h;
            alloc.release(r->off, r->bytes);
            active.erase(std::find(active.begin(), active.end(), r));
            if (r->status == LA_OK)
                stats.completed++;
            else
                stats.failed++;
        }
        cv.notify_all();
    }
    std::lock_guard<std::mutex> g(mu);
    stats.ticks++;
    stats.busy_seconds += now_s() - t0;
    stats.active = (int)active.size();
}

void la_server::run()
{
    if (hipSetDevice(device) != hipSuccess) {
        // nothing can run on this thread: the server stops as after a device
        // error (submit refuses new requests), and each request already queued
        // ends with LA_ERR_DEVICE
        std::unique_lock<std::mutex> g(mu);
        fatal = LA_ERR_DEVICE;
        for (;;) {
            for (Req *r : queue) {
                r->status = LA_ERR_DEVICE;
                r->state = DONE;
                r->t_done = now_s();
                stats.failed++;
            }
            queue.clear();
            cv.notify_all();
            cv.wait(g, [&] { return stop || !queue.empty(); });
            if (stop)
                return;
        }
    }
    for (;;) {
        {
            std::unique_lock<std::mutex> g(mu);
            cv.wait(g, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop)
                return;
        }
        tick();
    }
}

extern "C" {

la_status la_serve_create(la_context *ctx, const la_serve_config *cfg, void *arena,
                          size_t arena_bytes, la_server **out)
{
    if (out)
        *out = nullptr;
    if (!ctx || !arena || !out) {
        set_error("la_serve_create: NULL argument");
        return LA_ERR_INVALID_ARG;
    }
    if (((uintptr_t)arena & (kAlign - 1)) != 0) {
        set_error("la_serve_create: arena must be 256-byte aligned");
        return LA_ERR_INVALID_ARG;
    }
    if (arena_bytes < kReserve + (64u << 20)) {
        set_error("la_serve_create: arena of %zu bytes is below the %zu-byte minimum",
                  arena_bytes, kReserve + (64u << 20));
        return LA_ERR_OUT_OF_MEMORY;
    }
    std::unique_ptr<la_server> s(new (std::nothrow) la_server);
    if (!s) {
        set_error("la_serve_create: out of host memory");
        return LA_ERR_OUT_OF_MEMORY;
    }
    s->ctx = ctx;
    s->device = ctx->device;
    if (cfg && cfg->max_slots > 0)
        s->max_slots = std::min(cfg->max_slots, 4096);
    if (cfg && cfg->max_queue > 0)
        s->max_queue = cfg->max_queue;
    s->arena = (char *)arena;
    s->arena_bytes = arena_bytes;
    s->alloc.init(kReserve, arena_bytes & ~(kAlign - 1));
    hipError_t e = hipSetDevice(s->device);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&s->h_stage, kReserve, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&s->h_deltas, 4096 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        if (s->stream)
            (void)hipStreamDestroy(s->stream);
        if (s->h_stage)
            (void)hipHostFree(s->h_stage);
        set_error("la_serve_create: %s", hipGetErrorString(e));
        return LA_ERR_DEVICE;
    }
    la_server *raw = s.release();
    raw->worker = std::thread([raw] { raw->run(); });
    *out = raw;
    return LA_OK;
}

la_status la_serve_submit(la_server *s, int64_t m, int64_t n, const float *A_host, int64_t lda,
                          const la_polar_opts *opts, uint64_t *req_id)
{
    if (!s || !A_host || !req_id) {
        set_error("la_serve_submit: NULL argument");
        return LA_ERR_INVALID_ARG;
    }
    PolarPlan plan;
    la_status st = polar_plan(m, n, opts, &plan);
    if (st != LA_OK)
        return st;
    if (lda < n) {
        set_error("la_serve_submit: lda < n");
        return LA_ERR_SHAPE;
    }
    const size_t fp = footprint(m, n);
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->fatal != LA_OK) {
            set_error("la_serve_submit: server stopped after a device error");
            return s->fatal;
        }
        if (fp > s->alloc.capacity()) {
            set_error("la_serve_submit: request needs %zu bytes, arena holds %zu", fp,
                      s->alloc.capacity());
            return LA_ERR_TOO_LARGE;
        }
        if ((int)s->queue.size() >= s->max_queue) {
            set_error("la_serve_submit: queue full (%d)", s->max_queue);
            return LA_ERR_QUEUE_FULL;
        }
    }
    std::unique_ptr<Req> r(new (std::nothrow) Req);
    if (!r) {
        set_error("la_serve_submit: out of host memory");
        return LA_ERR_OUT_OF_MEMORY;
    }
    r->m = m;
    r->n = n;
    r->plan = plan;
    r->bytes = fp;
    r->info.last_delta = INFINITY;
    r->info.stop_reason = 2;
    const size_t mn = (size_t)m * n;
    hipError_t e = hipHostMalloc((void **)&r->io_pinned, mn * 4, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&r->h_pinned, (size_t)n * n * 4, hipHostMallocDefault);
    if (e != hipSuccess) {
        if (r->io_pinned) (void)hipHostFree(r->io_pinned);
        set_error("la_serve_submit: pinned allocation failed: %s", hipGetErrorString(e));
        return LA_ERR_OUT_OF_MEMORY;
    }
    for (int64_t i = 0; i < m; ++i)
        memcpy(r->io_pinned + i * n, A_host + i * lda, (size_t)n * 4);
    r->t_submit = now_s();
    std::lock_guard<std::mutex> g(s->mu);
    r->id = s->next_id++;
    *req_id = r->id;
    s->queue.push_back(r.get());
    s->all.emplace(r->id, std::move(r));
    s->stats.submitted++;
    s->stats.queued = (int)s->queue.size();
    s->cv.notify_all();
    return LA_OK;
}

la_status la_serve_poll(la_server *s, uint64_t id, float *U_host, float *H_host,
                        la_polar_info *info, la_status *req_status)
{
    if (!s) {
        set_error("la_serve_poll: NULL server");
        return LA_ERR_INVALID_ARG;
    }
    std::unique_ptr<Req> r;
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->all.find(id);
        if (it == s->all.end()) {
            set_error("la_serve_poll: unknown request %llu", (unsigned long long)id);
            return LA_ERR_UNKNOWN_REQUEST;
        }
        if (it->second->state != DONE)
            return LA_ERR_NOT_READY;
        r = std::move(it->second);
        s->all.erase(it);
    }
    if (U_host && (r->status == LA_OK || r->status == LA_ERR_NOT_CONVERGED))
        memcpy(U_host, r->io_pinned, (size_t)r->m * r->n * 4);
    if (H_host && (r->status == LA_OK || r->status == LA_ERR_NOT_CONVERGED))
        memcpy(H_host, r->h_pinned, (size_t)r->n * r->n * 4);
    if (info)
        *info = r->info;
    if (req_status)
        *req_status = r->status;
    if (r->io_pinned) (void)hipHostFree(r->io_pinned);
    if (r->h_pinned) (void)hipHostFree(r->h_pinned);
    return LA_OK;
}

la_status la_serve_stats_get(la_server *s, la_serve_stats *out)
{
    if (!s || !out) {
        set_error("la_serve_stats_get: NULL argument");
        return LA_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    return LA_OK;
}

la_status la_serve_destroy(la_server *s)
{
    if (!s)
        return LA_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable())
        s->worker.join();
    // teardown: an error here has no caller to act on it
    (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->all) {
        Req *r = kv.second.get();
        if (r->io_pinned) (void)hipHostFree(r->io_pinned);
        if (r->h_pinned) (void)hipHostFree(r->h_pinned);
    }
    (void)hipStreamDestroy(s->stream);
    (void)hipHostFree(s->h_stage);
    (void)hipHostFree(s->h_deltas);
    delete s;
    return LA_OK;
}

}  // extern "C"
