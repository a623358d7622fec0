// serve_core.h -- host side of the continuous-batching polar server: request
// registry, FIFO queue, admission by arena footprint, slots and per-tick
// staging capacity, the per-tick advance of every active request by one step
// of Algorithm NS_Polar (section III.D) with its stop test, completion,
// failure handling and statistics.  Plain C++17 with no HIP: the device work
// of a tick is delegated to an executor, so the same scheduler runs with the
// HIP executor of la_serve.hip and with a scripted executor on the CPU
// (tests), where it can be built with thread and address sanitizers.
//
// Executor interface (duck-typed; every call is made by the scheduler thread
// unless stated):
//   bool bind();                              // once, on the scheduler thread
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
};

template <class Exec>
class Core {
  public:
    Core(Exec &ex, const Config &cfg) : ex_(ex), cfg_(cfg)
    {
        alloc_.init(0, ex_.capacity());
    }
    ~Core() { shutdown(); }

    void start()
    {
        worker_ = std::thread([this] { run(); });
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
        if (worker_.joinable())
            worker_.join();
        std::lock_guard<std::mutex> g(mu_);
        for (auto &kv : all_)
            ex_.drop(*kv.second);
        all_.clear();
        queue_.clear();
        active_.clear();
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
        r->info.last_delta = INFINITY;
        r->info.stop_reason = 2;
        r->bytes = ex_.footprint(*r);
        ex_.stage_need(*r, &r->descs, &r->items);
        {
            std::lock_guard<std::mutex> g(mu_);
            if (fatal_ != LA_OK) {
                set_error("la_serve_submit: server stopped after a device error");
                return fatal_;
            }
            if (r->bytes > alloc_.capacity() || r->descs > ex_.desc_capacity() ||
                r->items > ex_.item_capacity()) {
                set_error("la_serve_submit: request needs %zu arena bytes, %zu descriptors and "
                          "%zu tile items; the server holds %zu, %zu and %zu",
                          r->bytes, r->descs, r->items, alloc_.capacity(), ex_.desc_capacity(),
                          ex_.item_capacity());
                return LA_ERR_TOO_LARGE;
            }
            if ((int)queue_.size() >= cfg_.max_queue) {
                set_error("la_serve_submit: queue full (%d)", cfg_.max_queue);
                return LA_ERR_QUEUE_FULL;
            }
        }
        st = ex_.stage_input(*r, A, lda);
        if (st != LA_OK)
            return st;
        r->t_submit = now_s();
        std::lock_guard<std::mutex> g(mu_);
        if (fatal_ != LA_OK || stop_) {
            ex_.drop(*r);
            set_error("la_serve_submit: server stopped");
            return fatal_ != LA_OK ? fatal_ : LA_ERR_DEVICE;
        }
        r->id = next_id_++;
        *id = r->id;
        queue_.push_back(r.get());
        all_.emplace(r->id, std::move(r));
        stats_.submitted++;
        stats_.queued = (int)queue_.size();
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
        if (r->status == LA_OK || r->status == LA_ERR_NOT_CONVERGED)
            ex_.copy_out(*r, U, H);
        if (info)
            *info = r->info;
        if (req_status)
            *req_status = r->status;
        ex_.drop(*r);
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
        return (int)active_.size();
    }

  private:
    Exec &ex_;
    Config cfg_;
    Arena alloc_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Req *> queue_;
    std::vector<Req *> active_;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> all_;
    uint64_t next_id_ = 1;
    bool stop_ = false, stopped_ = false;
    la_status fatal_ = LA_OK;
    la_serve_stats stats_{};
    size_t descs_used_ = 0, items_used_ = 0;   // staging of the active requests
    std::thread worker_;

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
    void fail_queue_locked()
    {
        const double t = now_s();
        for (Req *r : queue_)
            complete_locked(r, fatal_, t);
        queue_.clear();
        stats_.queued = 0;
        cv_.notify_all();
    }

    void run()
    {
        if (!ex_.bind()) {
            std::unique_lock<std::mutex> g(mu_);
            fatal_ = LA_ERR_DEVICE;
            for (;;) {
                fail_queue_locked();
                cv_.wait(g, [&] { return stop_ || !queue_.empty(); });
                if (stop_)
                    return;
            }
        }
        for (;;) {
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&] { return stop_ || !queue_.empty() || !active_.empty(); });
                if (stop_)
                    return;
                if (fatal_ != LA_OK) {
                    fail_queue_locked();
                    continue;
                }
            }
            tick();
        }
    }

    void tick()
    {
        const double t0 = now_s();
        std::vector<Req *> fresh, run;
        {
            // admission: FIFO while a slot, the arena and the tick's staging
            // hold the request
            std::lock_guard<std::mutex> g(mu_);
            while (!queue_.empty() && (int)active_.size() < cfg_.max_slots) {
                Req *r = queue_.front();
                if (descs_used_ + r->descs > ex_.desc_capacity() ||
                    items_used_ + r->items > ex_.item_capacity())
                    break;
                size_t off;
                if (!alloc_.alloc(r->bytes, &off))
                    break;
                queue_.pop_front();
                r->off = off;
                r->state = ACTIVE;
                descs_used_ += r->descs;
                items_used_ += r->items;
                ex_.place(*r, off);
                active_.push_back(r);
                fresh.push_back(r);
            }
            stats_.queued = (int)queue_.size();
            stats_.active = (int)active_.size();
            stats_.arena_high_water = alloc_.high_water();
            for (Req *r : active_)
                if (!r->finished)
                    run.push_back(r);
        }
        std::vector<double> fro2(fresh.size(), 0.0), delta2;
        la_status st = run.empty() && fresh.empty() ? LA_OK : ex_.tick(fresh, run, fro2, delta2);
        if (st != LA_OK) {
            std::lock_guard<std::mutex> g(mu_);
            fatal_ = LA_ERR_DEVICE;
            for (Req *r : active_) {
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
        for (Req *r : active_)     // only this thread changes active_
            if (r->finished)
                done.push_back(r);
        if (!done.empty()) {
            std::vector<Req *> ok;
            for (Req *r : done)
                if (r->status == LA_OK || r->status == LA_ERR_NOT_CONVERGED)
                    ok.push_back(r);
            la_status fs = (st == LA_OK && !ok.empty()) ? ex_.finish(ok) : LA_OK;
            const double t1 = now_s();
            std::lock_guard<std::mutex> g(mu_);
            if (fs != LA_OK)
                fatal_ = LA_ERR_DEVICE;
            for (Req *r : done) {
                la_status rs = r->status;
                if (fs != LA_OK && (rs == LA_OK || rs == LA_ERR_NOT_CONVERGED))
                    rs = LA_ERR_DEVICE;
                ex_.retire(*r);
                complete_locked(r, rs, t1);
                alloc_.release(r->off, r->bytes);
                descs_used_ -= r->descs;
                items_used_ -= r->items;
                active_.erase(std::find(active_.begin(), active_.end(), r));
            }
            cv_.notify_all();
        }
        std::lock_guard<std::mutex> g(mu_);
        stats_.ticks++;
        stats_.busy_seconds += now_s() - t0;
        stats_.active = (int)active_.size();
        if (fatal_ != LA_OK)
            fail_queue_locked();
    }
};

}  // namespace serve
}  // namespace la
