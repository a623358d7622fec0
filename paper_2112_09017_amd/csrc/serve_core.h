// serve_core.h -- host side of the continuous-batching polar server: request
// registry, FIFO queues, admission by arena footprint, slots and per-tick
// staging capacity, the per-tick advance of every active request by one step
// of Algorithm NS_Polar (section III.D) with its stop test, completion,
// failure handling and statistics.  Requests are routed by size (m n^2) to
// bands; each band has an executor and a scheduler thread of its own and
// ticks independently of the others, while the arena, the slots and the
// order of admission are shared.  Plain C++17 with no HIP: the device work
// of a tick is delegated to an executor, so the same scheduler runs with the
// HIP executor of la_serve.hip and with a scripted executor on the CPU
// (tests), where it can be built with thread and address sanitizers.
//
// Executor interface (duck-typed; every call is made by the scheduler thread
// of the executor's band unless stated):
//   bool bind();                              // once, on that thread
//   size_t capacity();                        // arena bytes requests may use
//   size_t footprint(const Req &);            // arena bytes of one request
//   void stage_need(const Req &, size_t *descs, size_t *items);
//                                             // per-tick staging of one request
//   size_t desc_capacity(), item_capacity();  // staging per tick
//   la_status stage_input(Req &, const float *A, int64_t lda);
//                                             // submit thread: host copy of A
//   void drop(Req &);                         // any thread: free host staging
//   void place(Req &, size_t off);            // device state at arena offset
//   la_status tick(const std::vector<Req *> &fresh, const std::vector<Req *> &run,
//                  std::vector<double> &fro2, std::vector<double> &delta2);
//       fresh: admitted this tick (input upload, ||A||_F^2, X0 = A / ||A||_F);
//       run: every request to advance by one step (the fresh ones included);
//       fro2[i]: ||A||_F^2 of fresh[i]; delta2[j]: ||U' - U||_F^2 of the j-th
//       request of `run` that takes a Newton-Schulz step.  Non-OK: a device
//       error (every active request fails, the server stops).
//   la_status finish(const std::vector<Req *> &done);
//       H and the results of the finished requests with status OK or
//       NOT_CONVERGED, ready for copy_out on return.
//   void retire(Req &);                       // the request left the arena
//   void copy_out(const Req &, float *U, float *H);   // poll thread
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "polar_host.h"

namespace la {
namespace serve {

inline double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// One entry of a grouped launch's item list: a tile of a problem, or empty
// (prob < 0).
struct Slot {
    int prob;
    int tile;
};

// Item list of a grouped launch for a device that deals workgroups to its
// XCDs in turn (workgroup b to XCD b % xcds, each XCD with its own L2): entry
// xcds i + x is the i-th item of XCD x.  Problem p has tiles[p] tiles (in
// linear order, neighbours sharing operand panels) of cost[p] each (its K).
// Every problem's tiles are cut into xcds contiguous runs, one per XCD, so
// each XCD holds an equal share of every problem and neighbouring tiles meet
// in one L2 (in plain order the tiles in flight on an XCD were every xcds-th
// tile of a problem); the runs one tile longer go to the XCDs with the least
// work so far, and an XCD takes the problems in order of decreasing cost.  The
// lists are padded to one length with empty entries: fewer than xcds per
// problem.
inline std::vector<Slot> xcd_layout(const std::vector<int64_t> &tiles,
                                    const std::vector<int64_t> &cost, int xcds)
{
    const int np = (int)tiles.size();
    std::vector<int> byk(np);
    for (int p = 0; p < np; ++p)
        byk[p] = p;
    std::stable_sort(byk.begin(), byk.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<std::vector<Slot>> lists(xcds);
    std::vector<double> load(xcds, 0.0);
    std::vector<int> ord(xcds);
    std::vector<int64_t> len(xcds);
    for (int p : byk) {
        const int64_t q = tiles[p] / xcds, r = tiles[p] % xcds;
        for (int x = 0; x < xcds; ++x)
            ord[x] = x;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return load[x] < load[y]; });
        for (int j = 0; j < xcds; ++j)
            len[ord[j]] = q + (j < r ? 1 : 0);
        int t = 0;
        for (int x = 0; x < xcds; ++x) {
            for (int64_t k = 0; k < len[x]; ++k)
                lists[x].push_back(Slot{p, t++});
            load[x] += (double)len[x] * (double)cost[p];
        }
    }
    size_t longest = 0;
    for (const auto &l : lists)
        longest = std::max(longest, l.size());
    std::vector<Slot> out(longest * xcds, Slot{-1, 0});
    for (int x = 0; x < xcds; ++x)
        for (size_t i = 0; i < lists[x].size(); ++i)
            out[i * xcds + x] = lists[x][i];
    return out;
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
    size_t used() const { return used_; }
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
    size_t free_blocks() const { return free_.size(); }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, high_ = 0, cap_ = 0;
};

enum State { QUEUED, ACTIVE, DONE };

struct Req {
    uint64_t id = 0;
    int64_t m = 0, n = 0;
    PolarPlan plan{};
    State state = QUEUED;
    la_status status = LA_OK;
    size_t off = 0, bytes = 0;         // arena block
    size_t descs = 0, items = 0;       // staging per tick
    int band = 0;                      // size band (scheduler thread and executor)
    StopState stop{};
    bool finished = false;             // no more steps
    la_polar_info info{};
    double t_submit = 0, t_done = 0;
    void *x = nullptr;                 // executor state
    bool precond() const { return info.iters_precond < plan.k_pre; }
    // precision of the next step: the plan's per phase, BF16X6 for the polish
    int step_prec() const
    {
        return precond() ? plan.prec_pre : (stop.stopped ? (int)PREC_BF16X6 : plan.prec_ns);
    }
};

struct Config {
    int max_slots = 32;
    int max_queue = 4096;
    // Size bands: a request with m n^2 <= band_work[i] (the first such i)
    // ticks in band i, a larger one in the last band.  Each band has an
    // executor and a scheduler thread of its own, so a small request's ticks
    // do not wait for a large request's steps.  One entry fewer than bands.
    std::vector<double> band_work;
};

template <class Exec>
class Core {
  public:
    // One executor per band (at least one); every executor reports the same
    // capacity(), the bytes of the arena area that all bands share.
    Core(const std::vector<Exec *> &bands, const Config &cfg) : cfg_(cfg)
    {
        for (Exec *e : bands) {
            bands_.emplace_back(new Band);
            bands_.back()->ex = e;
        }
        alloc_.init(0, bands_[0]->ex->capacity());
    }
    Core(Exec &ex, const Config &cfg) : Core(std::vector<Exec *>{&ex}, cfg) {}
    ~Core() { shutdown(); }

    void start()
    {
        for (size_t b = 0; b < bands_.size(); ++b)
            bands_[b]->worker = std::thread([this, b] { run(*bands_[b]); });
    }

    // Stops the scheduler; requests not yet polled are dropped.
    void shutdown()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            if (stopped_)
                return;
            stop_ = true;
            cv_.notify_all();
        }
        for (auto &b : bands_)
            if (b->worker.joinable())
                b->worker.join();
        std::lock_guard<std::mutex> g(mu_);
        for (auto &kv : all_)
            bands_[kv.second->band]->ex->drop(*kv.second);
        all_.clear();
        for (auto &b : bands_) {
            b->queue.clear();
            b->active.clear();
        }
        queued_ = active_ = 0;
        stopped_ = true;
    }

    la_status submit(int64_t m, int64_t n, const float *A, int64_t lda, const la_polar_opts *opts,
                     uint64_t *id)
    {
        if (!A || !id) {
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
        std::unique_ptr<Req> r(new (std::nothrow) Req);
        if (!r) {
            set_error("la_serve_submit: out of host memory");
            return LA_ERR_OUT_OF_MEMORY;
        }
        r->m = m;
        r->n = n;
        r->plan = plan;
        r->band = band_of(m, n);
        r->info.last_delta = INFINITY;
        r->info.stop_reason = 2;
        Band &B = *bands_[r->band];
        r->bytes = B.ex->footprint(*r);
        B.ex->stage_need(*r, &r->descs, &r->items);
        {
            std::lock_guard<std::mutex> g(mu_);
            if (fatal_ != LA_OK) {
                set_error("la_serve_submit: server stopped after a device error");
                return fatal_;
            }
            if (r->bytes > alloc_.capacity() || r->descs > B.ex->desc_capacity() ||
                r->items > B.ex->item_capacity()) {
                set_error("la_serve_submit: request needs %zu arena bytes, %zu descriptors and "
                          "%zu tile items; the server holds %zu, %zu and %zu",
                          r->bytes, r->descs, r->items, alloc_.capacity(), B.ex->desc_capacity(),
                          B.ex->item_capacity());
                return LA_ERR_TOO_LARGE;
            }
            if (queued_ >= cfg_.max_queue) {
                set_error("la_serve_submit: queue full (%d)", cfg_.max_queue);
                return LA_ERR_QUEUE_FULL;
            }
        }
        st = B.ex->stage_input(*r, A, lda);
        if (st != LA_OK)
            return st;
        r->t_submit = now_s();
        std::lock_guard<std::mutex> g(mu_);
        if (fatal_ != LA_OK || stop_) {
            B.ex->drop(*r);
            set_error("la_serve_submit: server stopped");
            return fatal_ != LA_OK ? fatal_ : LA_ERR_DEVICE;
        }
        r->id = next_id_++;
        *id = r->id;
        B.queue.push_back(r.get());
        all_.emplace(r->id, std::move(r));
        ++queued_;
        ++gen_;
        stats_.submitted++;
        stats_.queued = queued_;
        cv_.notify_all();
        return LA_OK;
    }

    la_status poll(uint64_t id, float *U, float *H, la_polar_info *info, la_status *req_status)
    {
        std::unique_ptr<Req> r;
        {
            std::lock_guard<std::mutex> g(mu_);
            auto it = all_.find(id);
            if (it == all_.end()) {
                set_error("la_serve_poll: unknown request %llu", (unsigned long long)id);
                return LA_ERR_UNKNOWN_REQUEST;
            }
            if (it->second->state != DONE)
                return LA_ERR_NOT_READY;
            r = std::move(it->second);
            all_.erase(it);
        }
        Exec &ex = *bands_[r->band]->ex;
        if (r->status == LA_OK || r->status == LA_ERR_NOT_CONVERGED)
            ex.copy_out(*r, U, H);
        if (info)
            *info = r->info;
        if (req_status)
            *req_status = r->status;
        ex.drop(*r);
        return LA_OK;
    }

    la_serve_stats stats()
    {
        std::lock_guard<std::mutex> g(mu_);
        return stats_;
    }

    // Requests in flight (tests).
    int active_count()
    {
        std::lock_guard<std::mutex> g(mu_);
        return active_;
    }

  private:
    struct Band {
        Exec *ex = nullptr;
        std::deque<Req *> queue;
        std::vector<Req *> active;     // changed by this band's thread only
        size_t descs_used = 0, items_used = 0;   // staging of the active requests
        std::thread worker;
    };

    Config cfg_;
    std::vector<std::unique_ptr<Band>> bands_;
    Arena alloc_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> all_;
    uint64_t next_id_ = 1;
    int queued_ = 0, active_ = 0;      // over all bands
    int in_tick_ = 0;                  // bands inside a tick
    uint64_t gen_ = 0;                 // bumped when a request arrives or leaves
    double busy_t0_ = 0;
    bool stop_ = false, stopped_ = false;
    la_status fatal_ = LA_OK;
    la_serve_stats stats_{};

    int band_of(int64_t m, int64_t n) const
    {
        const double w = (double)m * (double)n * (double)n;
        const int last = (int)bands_.size() - 1;
        for (int b = 0; b < last && b < (int)cfg_.band_work.size(); ++b)
            if (w <= cfg_.band_work[b])
                return b;
        return last;
    }

    // under mu_: request r leaves the server with status st
    void complete_locked(Req *r, la_status st, double t)
    {
        r->status = st;
        r->state = DONE;
        r->t_done = t;
        r->info.prec_precond = r->plan.prec_pre;
        r->info.prec_ns = r->plan.prec_ns;
        r->info.prec_h = r->plan.prec_h;
        if (st == LA_OK)
            stats_.completed++;
        else
            stats_.failed++;
    }

    // under mu_: every queued request fails with the server's fatal status
    void fail_queues_locked()
    {
        const double t = now_s();
        for (auto &b : bands_) {
            for (Req *r : b->queue)
                complete_locked(r, fatal_, t);
            b->queue.clear();
        }
        queued_ = 0;
        stats_.queued = 0;
        cv_.notify_all();
    }

    // under mu_, on B's thread: B's active requests fail with the fatal status
    // (a device error in another band)
    void fail_active_locked(Band &B)
    {
        const double t = now_s();
        for (Req *r : B.active) {
            B.ex->retire(*r);
            complete_locked(r, fatal_, t);
            alloc_.release(r->off, r->bytes);
        }
        active_ -= (int)B.active.size();
        if (!B.active.empty())
            ++gen_;
        B.active.clear();
        B.descs_used = B.items_used = 0;
        stats_.active = active_;
        cv_.notify_all();
    }

    bool any_queued_locked() const { return queued_ > 0; }

    void run(Band &B)
    {
        if (!B.ex->bind()) {
            std::unique_lock<std::mutex> g(mu_);
            fatal_ = LA_ERR_DEVICE;
            for (;;) {
                fail_queues_locked();
                cv_.wait(g, [&] { return stop_ || any_queued_locked(); });
                if (stop_)
                    return;
            }
        }
        // A band with requests in flight ticks back to back; one whose queue
        // is held up (arena or slots taken by the other band, or an older
        // request there) waits until a request arrives or leaves.
        uint64_t seen = ~(uint64_t)0;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&] {
                    return stop_ || !B.active.empty() || (!B.queue.empty() && gen_ != seen) ||
                           (fatal_ != LA_OK && any_queued_locked());
                });
                if (stop_)
                    return;
                if (fatal_ != LA_OK) {
                    fail_active_locked(B);
                    fail_queues_locked();
                    continue;
                }
                seen = gen_;
            }
            tick(B);
        }
    }

    // under mu_: admission of B's queued requests, FIFO within the band, while
    // a slot, the arena and the band's staging hold the request.  Across
    // bands the order of submission is kept for the arena and the slots: a
    // request is admitted only if the older requests at the heads of the
    // other bands' queues would still find room.
    void admit_locked(Band &B, std::vector<Req *> &fresh)
    {
        while (!B.queue.empty() && active_ < cfg_.max_slots) {
            Req *r = B.queue.front();
            if (B.descs_used + r->descs > B.ex->desc_capacity() ||
                B.items_used + r->items > B.ex->item_capacity())
                break;
            size_t held = 0;
            int held_slots = 0;
            for (auto &o : bands_)
                if (o.get() != &B && !o->queue.empty() && o->queue.front()->id < r->id) {
                    held += o->queue.front()->bytes;
                    ++held_slots;
                }
            if (active_ + 1 + held_slots > cfg_.max_slots)
                break;
            if (held && alloc_.capacity() - alloc_.used() < r->bytes + held)
                break;
            size_t off;
            if (!alloc_.alloc(r->bytes, &off))
                break;
            B.queue.pop_front();
            --queued_;
            r->off = off;
            r->state = ACTIVE;
            B.descs_used += r->descs;
            B.items_used += r->items;
            B.ex->place(*r, off);
            B.active.push_back(r);
            ++active_;
            fresh.push_back(r);
        }
        stats_.queued = queued_;
        stats_.active = active_;
        stats_.arena_high_water = alloc_.high_water();
    }

    void tick(Band &B)
    {
        Exec &ex = *B.ex;
        std::vector<Req *> fresh, run;
        {
            std::lock_guard<std::mutex> g(mu_);
            if (in_tick_++ == 0)
                busy_t0_ = now_s();
            admit_locked(B, fresh);
            for (Req *r : B.active)
                if (!r->finished)
                    run.push_back(r);
        }
        const bool work = !run.empty() || !fresh.empty();
        std::vector<double> fro2(fresh.size(), 0.0), delta2;
        la_status st = work ? ex.tick(fresh, run, fro2, delta2) : LA_OK;
        if (st != LA_OK) {
            std::lock_guard<std::mutex> g(mu_);
            fatal_ = LA_ERR_DEVICE;
            for (Req *r : B.active) {
                r->status = LA_ERR_DEVICE;
                r->finished = true;
            }
        } else {
            for (size_t i = 0; i < fresh.size(); ++i) {
                const double fro = sqrt(fro2[i]);
                fresh[i]->info.fro_norm_a = fro;
                if (!(fro > 0.0) || !isfinite(fro)) {
                    fresh[i]->status = LA_ERR_NONFINITE;
                    fresh[i]->finished = true;
                }
            }
            size_t k = 0;
            for (Req *r : run) {
                const bool ns = !r->precond();
                const double d2 = ns ? delta2[k++] : 0.0;
                if (r->finished)       // failed at admission (norm): its step is discarded
                    continue;
                if (!ns) {
                    r->info.iters_precond++;
                    continue;
                }
                r->info.iters_ns++;
                const double delta = sqrt(d2);
                r->info.last_delta = delta;
                if (!isfinite(delta)) {
                    r->status = LA_ERR_NONFINITE;
                    r->finished = true;
                    continue;
                }
                const StopDecision dcs = stop_test(r->plan, r->m, r->n, delta, r->stop,
                                                   r->info.iters_ns);
                r->info.stop_reason = r->stop.reason;
                if (dcs == STOP_DONE) {
                    r->finished = true;
                } else if (dcs == STOP_CAP) {
                    r->status = LA_ERR_NOT_CONVERGED;
                    r->finished = true;
                }
            }
        }
        std::vector<Req *> done;
        for (Req *r : B.active)     // only this thread changes B.active
            if (r->finished)
                done.push_back(r);
        if (!done.empty()) {
            std::vector<Req *> ok;
            for (Req *r : done)
                if (r->status == LA_OK || r->status == LA_ERR_NOT_CONVERGED)
                    ok.push_back(r);
            la_status fs = (st == LA_OK && !ok.empty()) ? ex.finish(ok) : LA_OK;
            const double t1 = now_s();
            std::lock_guard<std::mutex> g(mu_);
            if (fs != LA_OK)
                fatal_ = LA_ERR_DEVICE;
            for (Req *r : done) {
                la_status rs = r->status;
                if (fs != LA_OK && (rs == LA_OK || rs == LA_ERR_NOT_CONVERGED))
                    rs = LA_ERR_DEVICE;
                ex.retire(*r);
                complete_locked(r, rs, t1);
                alloc_.release(r->off, r->bytes);
                B.descs_used -= r->descs;
                B.items_used -= r->items;
                B.active.erase(std::find(B.active.begin(), B.active.end(), r));
                --active_;
            }
            ++gen_;
            cv_.notify_all();
        }
        std::lock_guard<std::mutex> g(mu_);
        if (work)
            stats_.ticks++;
        if (--in_tick_ == 0)
            stats_.busy_seconds += now_s() - busy_t0_;
        stats_.active = active_;
        if (fatal_ != LA_OK)
            fail_queues_locked();
    }
};

}  // namespace serve
}  // namespace la
