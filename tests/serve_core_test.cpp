// CPU tests of the serving scheduler (paper_2112_09017_amd/csrc/serve_core.h)
// against a scripted executor: no GPU, built with g++ and run under thread and
// address sanitizers by tests/test_serve_core_cpu.py.
//
// The fake executor keeps each request's "singular values" (the absolute
// diagonal of its input, normalised by their 2-norm) and moves them through
// the scalar maps of Algorithm NS_Polar: the preconditioning polynomial of
// eqs. (a_def)-(RogueScalar) and the Newton-Schulz map of eq. (NS_scalar).  A
// tick reports ||A||_F^2 of the admitted requests and, for every
// Newton-Schulz step, the step norm of that spectrum.  The result of a request
// is A / ||A||_F, so a mix-up between requests shows.  Failures are injected
// on demand: a device error at a given tick or in finish, a failing bind, and
// a refused host staging.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <cmath>
#include <functional>
#include <set>
#include <string>
#include <vector>

#include "serve_core.h"

namespace la {
static thread_local char g_err[512];
void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}
}  // namespace la

using namespace la;
using namespace la::serve;

static int g_fail = 0;
#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            fprintf(stderr, "%s:%d: CHECK failed: %s (%s)\n", __FILE__, __LINE__, #c, \
                    la::g_err);                                                    \
            ++g_fail;                                                              \
        }                                                                          \
    } while (0)

struct FakeState {
    std::vector<float> A;      // staged input
    std::vector<double> x;     // spectrum of the iterate
    std::vector<float> U;      // result
    int64_t m = 0, n = 0;
};

// Observations shared by the executors of a core's size bands.
struct Obs {
    std::mutex mu;
    std::map<size_t, size_t> blocks;   // offset -> bytes of active requests
    bool overlap = false;
    std::vector<uint64_t> admitted;
    int live = 0, max_live = 0;
};

struct Fake {
    Obs *obs = nullptr;         // shared with the other bands' executors
    size_t cap = 1 << 20;
    size_t dcap = 64, icap = 4096;
    bool bind_ok = true;
    int fail_tick = -1;         // device error in this tick (0-based)
    bool fail_finish = false;
    uint64_t refuse_stage_n = 0;  // stage_input of an n x n request with this n fails
    std::function<void()> gate;   // called at the start of every tick
    // observations
    std::mutex mu;
    int ticks = 0;
    int max_active = 0;
    std::vector<uint64_t> admitted;
    std::map<size_t, size_t> blocks;   // offset -> bytes of active requests
    bool overlap = false, stage_over = false;
    std::set<Req *> live;

    bool bind() { return bind_ok; }
    size_t capacity() { return cap; }
    size_t footprint(const Req &r) { return (size_t)(3 * r.m * r.n + r.n * r.n) * 4; }
    void stage_need(const Req &r, size_t *d, size_t *i)
    {
        *d = 2;
        *i = (size_t)((r.n + 127) / 128) * ((r.m + 127) / 128) + (size_t)((r.n + 127) / 128);
    }
    size_t desc_capacity() { return dcap; }
    size_t item_capacity() { return icap; }
    la_status stage_input(Req &r, const float *A, int64_t lda)
    {
        if (refuse_stage_n && (uint64_t)r.n == refuse_stage_n) {
            set_error("fake: staging refused");
            return LA_ERR_OUT_OF_MEMORY;
        }
        FakeState *f = new FakeState;
        f->m = r.m;
        f->n = r.n;
        f->A.resize((size_t)r.m * r.n);
        for (int64_t i = 0; i < r.m; ++i)
            memcpy(&f->A[(size_t)i * r.n], A + i * lda, (size_t)r.n * 4);
        r.x = f;
        return LA_OK;
    }
    void drop(Req &r)
    {
        delete (FakeState *)r.x;
        r.x = nullptr;
    }
    void place(Req &r, size_t off)
    {
        std::lock_guard<std::mutex> g(mu);
        for (auto &b : blocks)
            if (off < b.first + b.second && b.first < off + r.bytes)
                overlap = true;
        blocks[off] = r.bytes;
        admitted.push_back(r.id);
        live.insert(&r);
        max_active = std::max(max_active, (int)live.size());
        if (obs) {
            std::lock_guard<std::mutex> o(obs->mu);
            for (auto &b : obs->blocks)
                if (off < b.first + b.second && b.first < off + r.bytes)
                    obs->overlap = true;
            obs->blocks[off] = r.bytes;
            obs->admitted.push_back(r.id);
            obs->max_live = std::max(obs->max_live, ++obs->live);
        }
    }
    la_status tick(const std::vector<Req *> &fresh, const std::vector<Req *> &run,
                   std::vector<double> &fro2, std::vector<double> &delta2)
    {
        if (gate)
            gate();
        int t;
        {
            std::lock_guard<std::mutex> g(mu);
            t = ticks++;
            size_t d = 0, it = 0;
            for (Req *r : live) {
                d += r->descs;
                it += r->items;
            }
            if (d > dcap || it > icap)
                stage_over = true;
        }
        if (t == fail_tick)
            return LA_ERR_DEVICE;
        for (size_t i = 0; i < fresh.size(); ++i) {
            FakeState *f = (FakeState *)fresh[i]->x;
            double s2 = 0.0;
            for (float v : f->A)
                s2 += (double)v * v;
            fro2[i] = s2;
            double d2 = 0.0;
            for (int64_t j = 0; j < f->n; ++j)
                d2 += (double)f->A[(size_t)j * f->n + j] * f->A[(size_t)j * f->n + j];
            f->x.assign((size_t)f->n, 0.0);
            for (int64_t j = 0; j < f->n; ++j)
                f->x[j] = std::fabs((double)f->A[(size_t)j * f->n + j]) / std::sqrt(d2);
        }
        for (Req *r : run) {
            FakeState *f = (FakeState *)r->x;
            if (r->precond()) {
                for (double &v : f->x)
                    v = r->plan.a * v * (1.0 - r->plan.c * v * v);
            } else {
                double d2 = 0.0;
                for (double &v : f->x) {
                    const double nv = 0.5 * v * (3.0 - v * v);
                    d2 += (nv - v) * (nv - v);
                    v = nv;
                }
                delta2.push_back(d2);
            }
        }
        return LA_OK;
    }
    la_status finish(const std::vector<Req *> &done)
    {
        if (fail_finish)
            return LA_ERR_DEVICE;
        for (Req *r : done) {
            FakeState *f = (FakeState *)r->x;
            f->U.resize(f->A.size());
            for (size_t i = 0; i < f->A.size(); ++i)
                f->U[i] = (float)((double)f->A[i] / r->info.fro_norm_a);
        }
        return LA_OK;
    }
    void retire(Req &r)
    {
        std::lock_guard<std::mutex> g(mu);
        blocks.erase(r.off);
        live.erase(&r);
        if (obs) {
            std::lock_guard<std::mutex> o(obs->mu);
            obs->blocks.erase(r.off);
            --obs->live;
        }
    }
    void copy_out(const Req &r, float *U, float *H)
    {
        FakeState *f = (FakeState *)r.x;
        if (U)
            memcpy(U, f->U.data(), f->U.size() * 4);
        if (H)
            for (int64_t i = 0; i < r.n * r.n; ++i)
                H[i] = 1.0f;
    }
};

// An n x n input with diagonal geometric from 1 down to 1/cond and a small
// off-diagonal pattern that depends on `tag`.
static std::vector<float> make_input(int64_t m, int64_t n, double cond, int tag)
{
    std::vector<float> A((size_t)m * n, 0.0f);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            A[(size_t)i * n + j] = 1e-3f * (float)(((i * 31 + j * 17 + tag * 7) % 13) - 6);
    for (int64_t j = 0; j < n; ++j)
        A[(size_t)j * n + j] = (float)std::pow(cond, -(double)j / std::max<int64_t>(1, n - 1));
    return A;
}

// The stop rule written out independently of the scheduler: steps of the
// scalar model until ||x' - x|| <= max(m, n) eps, the stagnation rule or the
// cap; returns (k_pre, k_ns, reason).
static void model(const std::vector<float> &A, int64_t m, int64_t n, const PolarPlan &p,
                  int *kp, int *kn, int *reason)
{
    std::vector<double> x(n);
    double d2 = 0.0;
    for (int64_t j = 0; j < n; ++j)
        d2 += (double)A[(size_t)j * n + j] * A[(size_t)j * n + j];
    for (int64_t j = 0; j < n; ++j)
        x[j] = std::fabs((double)A[(size_t)j * n + j]) / std::sqrt(d2);
    for (int k = 0; k < p.k_pre; ++k)
        for (double &v : x)
            v = p.a * v * (1.0 - p.c * v * v);
    *kp = p.k_pre;
    double prev = INFINITY;
    int steps = 0;
    bool stopped = false;
    *reason = 2;
    for (;;) {
        double s = 0.0;
        for (double &v : x) {
            const double nv = 0.5 * v * (3.0 - v * v);
            s += (nv - v) * (nv - v);
            v = nv;
        }
        ++steps;
        const double d = std::sqrt(s);
        if (stopped)
            break;   // polish step done
        if (d <= (double)std::max(m, n) * p.eps) {
            stopped = true;
            *reason = 0;
        } else if (p.stagnation && d < 1e-2 * std::sqrt((double)n) && d > 0.5 * prev) {
            stopped = true;
            *reason = 1;
        }
        prev = d;
        if (stopped && !p.polish)
            break;
        if (!stopped && steps >= p.max_iter)
            break;
    }
    *kn = steps;
}

struct Sub {
    uint64_t id;
    int64_t m, n;
    std::vector<float> A;
    la_polar_opts o;
};

static Sub submit_one(Core<Fake> &c, int64_t m, int64_t n, double cond, int tag,
                      la_polar_opts o = la_polar_opts{}, la_status expect = LA_OK)
{
    Sub s{0, m, n, make_input(m, n, cond, tag), o};
    const la_status st = c.submit(m, n, s.A.data(), n, &o, &s.id);
    CHECK(st == expect);
    return s;
}

static bool wait_done(Core<Fake> &c, Sub &s, la_status *rs, la_polar_info *info,
                      std::vector<float> *U, double timeout = 20.0)
{
    const double t0 = now_s();
    U->assign((size_t)s.m * s.n, NAN);
    std::vector<float> H((size_t)s.n * s.n);
    for (;;) {
        const la_status st = c.poll(s.id, U->data(), H.data(), info, rs);
        if (st == LA_OK)
            return true;
        CHECK(st == LA_ERR_NOT_READY);
        if (st != LA_ERR_NOT_READY || now_s() - t0 > timeout)
            return false;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

static void check_result(const Sub &s, la_status rs, const la_polar_info &info,
                         const std::vector<float> &U)
{
    PolarPlan p;
    CHECK(polar_plan(s.m, s.n, &s.o, &p) == LA_OK);
    int kp, kn, reason;
    model(s.A, s.m, s.n, p, &kp, &kn, &reason);
    CHECK(info.iters_precond == kp);
    CHECK(info.iters_ns == kn);
    CHECK(info.stop_reason == reason);
    CHECK(rs == (reason == 2 ? LA_ERR_NOT_CONVERGED : LA_OK));
    double s2 = 0.0;
    for (float v : s.A)
        s2 += (double)v * v;
    CHECK(std::fabs(info.fro_norm_a - std::sqrt(s2)) <= 1e-12 * std::sqrt(s2));
    bool same = true;   // the request's own result, not another's
    for (size_t i = 0; i < U.size(); ++i)
        same &= U[i] == (float)((double)s.A[i] / info.fro_norm_a);
    CHECK(same);
}

static void test_mix_and_counts()
{
    Fake f;
    Config cfg;
    cfg.max_slots = 8;
    Core<Fake> c(f, cfg);
    c.start();
    std::vector<Sub> subs;
    const int64_t sizes[][2] = {{8, 8}, {24, 16}, {16, 16}, {40, 12}, {12, 12}, {64, 32}};
    for (int i = 0; i < 18; ++i) {
        la_polar_opts o{};
        if (i % 5 == 3)
            o.polish = 1;
        if (i % 7 == 4)
            o.s_minus = 0.3;
        subs.push_back(submit_one(c, sizes[i % 6][0], sizes[i % 6][1], std::pow(10.0, 1 + i % 5),
                                  i, o));
    }
    for (Sub &s : subs) {
        la_status rs;
        la_polar_info info;
        std::vector<float> U;
        CHECK(wait_done(c, s, &rs, &info, &U));
        check_result(s, rs, info, U);
    }
    const la_serve_stats st = c.stats();
    CHECK(st.completed == subs.size() && st.failed == 0 && st.submitted == subs.size());
    CHECK(f.max_active <= cfg.max_slots && f.max_active > 1);
    CHECK(!f.overlap && !f.stage_over);
    // FIFO admission
    for (size_t i = 0; i < f.admitted.size(); ++i)
        CHECK(f.admitted[i] == subs[i].id);
    // a second poll: unknown
    la_status rs;
    CHECK(c.poll(subs[0].id, nullptr, nullptr, nullptr, &rs) == LA_ERR_UNKNOWN_REQUEST);
    printf("mix_and_counts: %llu ticks, max active %d\n", (unsigned long long)st.ticks,
           f.max_active);
}

static void test_arena_slots_and_staging()
{
    // arena holds two 16 x 16 requests (3 mn + n^2 floats = 4096 bytes each)
    {
        Fake f;
        f.cap = 2 * 4096 + 100;
        Config cfg;
        cfg.max_slots = 16;
        Core<Fake> c(f, cfg);
        c.start();
        std::vector<Sub> subs;
        for (int i = 0; i < 7; ++i)
            subs.push_back(submit_one(c, 16, 16, 1e3, i));
        submit_one(c, 64, 64, 10.0, 99, la_polar_opts{}, LA_ERR_TOO_LARGE);
        for (Sub &s : subs) {
            la_status rs;
            la_polar_info info;
            std::vector<float> U;
            CHECK(wait_done(c, s, &rs, &info, &U));
            check_result(s, rs, info, U);
        }
        CHECK(f.max_active == 2 && !f.overlap);
        printf("arena: max active %d\n", f.max_active);
    }
    // slots
    {
        Fake f;
        Config cfg;
        cfg.max_slots = 3;
        Core<Fake> c(f, cfg);
        c.start();
        std::vector<Sub> subs;
        for (int i = 0; i < 10; ++i)
            subs.push_back(submit_one(c, 12, 12, 1e2, i));
        for (Sub &s : subs) {
            la_status rs;
            la_polar_info info;
            std::vector<float> U;
            CHECK(wait_done(c, s, &rs, &info, &U));
        }
        CHECK(f.max_active == 3);
        printf("slots: max active %d\n", f.max_active);
    }
    // staging: each request takes 2 descriptors; 5 fit a 10-descriptor tick
    {
        Fake f;
        f.dcap = 10;
        Config cfg;
        cfg.max_slots = 64;
        Core<Fake> c(f, cfg);
        c.start();
        std::vector<Sub> subs;
        for (int i = 0; i < 20; ++i)
            subs.push_back(submit_one(c, 8, 8, 1e2, i));
        for (Sub &s : subs) {
            la_status rs;
            la_polar_info info;
            std::vector<float> U;
            CHECK(wait_done(c, s, &rs, &info, &U));
            check_result(s, rs, info, U);
        }
        CHECK(f.max_active == 5 && !f.stage_over);
        // one request's tile items beyond the tick's capacity: too large
        f.icap = 4;
        submit_one(c, 512, 512, 10.0, 1, la_polar_opts{}, LA_ERR_TOO_LARGE);
        printf("staging: max active %d\n", f.max_active);
    }
}

static void test_queue_full_and_gate()
{
    Fake f;
    std::mutex gm;
    std::condition_variable gcv;
    bool open = false;
    f.gate = [&] {
        std::unique_lock<std::mutex> g(gm);
        gcv.wait(g, [&] { return open; });
    };
    Config cfg;
    cfg.max_slots = 1;
    cfg.max_queue = 3;
    Core<Fake> c(f, cfg);
    c.start();
    std::vector<Sub> subs;
    subs.push_back(submit_one(c, 8, 8, 10.0, 0));
    // wait until the first is admitted (the tick is blocked in the gate)
    while (c.active_count() < 1)
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    for (int i = 1; i <= 3; ++i)
        subs.push_back(submit_one(c, 8, 8, 10.0, i));
    submit_one(c, 8, 8, 10.0, 9, la_polar_opts{}, LA_ERR_QUEUE_FULL);
    la_status rs;
    CHECK(c.poll(subs[1].id, nullptr, nullptr, nullptr, &rs) == LA_ERR_NOT_READY);
    {
        std::lock_guard<std::mutex> g(gm);
        open = true;
    }
    gcv.notify_all();
    for (Sub &s : subs) {
        la_polar_info info;
        std::vector<float> U;
        CHECK(wait_done(c, s, &rs, &info, &U));
        check_result(s, rs, info, U);
    }
    printf("queue_full: ok\n");
}

static void test_nonfinite_cap_and_errors()
{
    {
        Fake f;
        Config cfg;
        Core<Fake> c(f, cfg);
        c.start();
        Sub good = submit_one(c, 16, 16, 1e3, 1);
        Sub bad = submit_one(c, 16, 16, 1e3, 2);
        bad.A[5] = NAN;
        // resubmit the NaN input (the copy above was taken before the change)
        Sub bad2{0, 16, 16, bad.A, la_polar_opts{}};
        CHECK(c.submit(16, 16, bad2.A.data(), 16, nullptr, &bad2.id) == LA_OK);
        la_polar_opts capo{};
        capo.max_iter = 2;
        Sub capped = submit_one(c, 16, 16, 1e5, 3, capo);
        la_status rs;
        la_polar_info info;
        std::vector<float> U;
        CHECK(wait_done(c, good, &rs, &info, &U));
        check_result(good, rs, info, U);
        CHECK(wait_done(c, bad2, &rs, &info, &U));
        CHECK(rs == LA_ERR_NONFINITE);
        CHECK(wait_done(c, capped, &rs, &info, &U));
        CHECK(rs == LA_ERR_NOT_CONVERGED && info.iters_ns == 2 && info.stop_reason == 2);
        check_result(capped, rs, info, U);
        CHECK(wait_done(c, bad, &rs, &info, &U));
        CHECK(rs == LA_OK);
        // bad arguments
        uint64_t id;
        std::vector<float> A(64, 1.0f);
        CHECK(c.submit(4, 8, A.data(), 8, nullptr, &id) == LA_ERR_SHAPE);    // m < n
        CHECK(c.submit(8, 8, A.data(), 4, nullptr, &id) == LA_ERR_SHAPE);    // lda < n
        CHECK(c.submit(8, 8, nullptr, 8, nullptr, &id) == LA_ERR_INVALID_ARG);
        la_polar_opts bo{};
        bo.prec_ns = 9;
        CHECK(c.submit(8, 8, A.data(), 8, &bo, &id) == LA_ERR_INVALID_ARG);
        CHECK(c.poll(12345, nullptr, nullptr, nullptr, &rs) == LA_ERR_UNKNOWN_REQUEST);
        const la_serve_stats st = c.stats();
        CHECK(st.completed == 2 && st.failed == 2);   // NONFINITE and NOT_CONVERGED
    }
    {
        // refused host staging fails the submit only
        Fake f;
        f.refuse_stage_n = 24;
        Config cfg;
        Core<Fake> c(f, cfg);
        c.start();
        submit_one(c, 24, 24, 10.0, 1, la_polar_opts{}, LA_ERR_OUT_OF_MEMORY);
        Sub s = submit_one(c, 16, 16, 10.0, 2);
        la_status rs;
        la_polar_info info;
        std::vector<float> U;
        CHECK(wait_done(c, s, &rs, &info, &U));
        check_result(s, rs, info, U);
    }
    printf("nonfinite_cap_and_errors: ok\n");
}

static void test_device_errors()
{
    {
        // device error in the third tick: every active request fails, the
        // queued ones too, and later submits are refused
        Fake f;
        f.fail_tick = 2;
        std::atomic<bool> hold{true};
        Config cfg;
        cfg.max_slots = 2;
        Core<Fake> c(f, cfg);
        std::vector<Sub> subs;
        for (int i = 0; i < 5; ++i)
            subs.push_back(submit_one(c, 16, 16, 1e4, i));
        c.start();
        for (Sub &s : subs) {
            la_status rs;
            la_polar_info info;
            std::vector<float> U;
            CHECK(wait_done(c, s, &rs, &info, &U));
            CHECK(rs == LA_ERR_DEVICE);
        }
        uint64_t id;
        std::vector<float> A(64, 1.0f);
        CHECK(c.submit(8, 8, A.data(), 8, nullptr, &id) == LA_ERR_DEVICE);
        const la_serve_stats st = c.stats();
        CHECK(st.failed == 5 && st.completed == 0);
        (void)hold;
    }
    {
        Fake f;
        f.fail_finish = true;
        Config cfg;
        Core<Fake> c(f, cfg);
        c.start();
        Sub s = submit_one(c, 8, 8, 10.0, 1);
        la_status rs;
        la_polar_info info;
        std::vector<float> U;
        CHECK(wait_done(c, s, &rs, &info, &U));
        CHECK(rs == LA_ERR_DEVICE);
    }
    {
        Fake f;
        f.bind_ok = false;
        Config cfg;
        Core<Fake> c(f, cfg);
        Sub s = submit_one(c, 8, 8, 10.0, 1);
        c.start();
        la_status rs;
        la_polar_info info;
        std::vector<float> U;
        CHECK(wait_done(c, s, &rs, &info, &U));
        CHECK(rs == LA_ERR_DEVICE);
        uint64_t id;
        CHECK(c.submit(8, 8, s.A.data(), 8, nullptr, &id) == LA_ERR_DEVICE);
    }
    printf("device_errors: ok\n");
}

static void test_threads_and_shutdown()
{
    // several submitters and pollers at once, then shutdown with requests in
    // flight (the sanitizer builds check the locking)
    Fake f;
    Config cfg;
    cfg.max_slots = 6;
    Core<Fake> c(f, cfg);
    c.start();
    std::atomic<int> ok{0};
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t)
        th.emplace_back([&, t] {
            for (int i = 0; i < 12; ++i) {
                Sub s = submit_one(c, 12 + 8 * (i % 3), 8 + 4 * (i % 2), 1e2, 100 * t + i);
                la_status rs;
                la_polar_info info;
                std::vector<float> U;
                if (wait_done(c, s, &rs, &info, &U)) {
                    check_result(s, rs, info, U);
                    ++ok;
                }
                (void)c.stats();
            }
        });
    for (auto &x : th)
        x.join();
    CHECK(ok == 48);
    // leave some in flight and shut down
    for (int i = 0; i < 10; ++i)
        submit_one(c, 32, 32, 1e5, i);
    c.shutdown();
    printf("threads_and_shutdown: ok\n");
}

// Two size bands: 12 x 12 and 16 x 16 requests (m n^2 <= 16^3) in band 0,
// larger ones in band 1.
static Config band_cfg(int slots)
{
    Config cfg;
    cfg.max_slots = slots;
    cfg.band_work.push_back(16.0 * 16.0 * 16.0);
    return cfg;
}

static void test_bands_route_and_mix()
{
    Obs obs;
    Fake f0, f1;
    f0.obs = f1.obs = &obs;
    Config cfg = band_cfg(8);
    Core<Fake> c({&f0, &f1}, cfg);
    c.start();
    std::vector<Sub> subs;
    std::vector<uint64_t> small, large;
    const int64_t sizes[][2] = {{8, 8}, {24, 16}, {16, 16}, {40, 12}, {12, 12}, {64, 32}};
    for (int i = 0; i < 18; ++i) {
        const int64_t m = sizes[i % 6][0], n = sizes[i % 6][1];
        subs.push_back(submit_one(c, m, n, std::pow(10.0, 1 + i % 5), i));
        (m * n * n <= 16 * 16 * 16 ? small : large).push_back(subs.back().id);
    }
    for (Sub &s : subs) {
        la_status rs;
        la_polar_info info;
        std::vector<float> U;
        CHECK(wait_done(c, s, &rs, &info, &U));
        check_result(s, rs, info, U);
    }
    CHECK(f0.admitted == small);   // each band admits its own, in order
    CHECK(f1.admitted == large);
    CHECK(!obs.overlap && !f0.stage_over && !f1.stage_over);
    CHECK(obs.max_live <= cfg.max_slots && obs.live == 0);
    const la_serve_stats st = c.stats();
    CHECK(st.completed == subs.size() && st.failed == 0);
    CHECK(st.ticks == (uint64_t)(f0.ticks + f1.ticks));
    printf("bands_route_and_mix: %d + %d ticks, max active %d\n", f0.ticks, f1.ticks,
           obs.max_live);
}

// A band held inside a tick does not hold up the other band.
static void test_bands_tick_independently()
{
    Obs obs;
    Fake f0, f1;
    f0.obs = f1.obs = &obs;
    std::mutex gm;
    std::condition_variable gcv;
    bool open = false;
    f1.gate = [&] {
        std::unique_lock<std::mutex> g(gm);
        gcv.wait(g, [&] { return open; });
    };
    Core<Fake> c({&f0, &f1}, band_cfg(8));
    c.start();
    Sub big = submit_one(c, 32, 32, 1e4, 1);
    while (c.active_count() < 1)
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    std::vector<Sub> subs;
    for (int i = 0; i < 6; ++i)
        subs.push_back(submit_one(c, 12, 12, 1e3, 10 + i));
    for (Sub &s : subs) {
        la_status rs;
        la_polar_info info;
        std::vector<float> U;
        CHECK(wait_done(c, s, &rs, &info, &U));
        check_result(s, rs, info, U);
    }
    la_status rs;
    CHECK(c.poll(big.id, nullptr, nullptr, nullptr, &rs) == LA_ERR_NOT_READY);
    {
        std::lock_guard<std::mutex> g(gm);
        open = true;
    }
    gcv.notify_all();
    la_polar_info info;
    std::vector<float> U;
    CHECK(wait_done(c, big, &rs, &info, &U));
    check_result(big, rs, info, U);
    printf("bands_tick_independently: ok\n");
}

// No request overtakes an older one of the other band for the arena or for
// a slot: S1 (band 0) holds what B (band 1) needs; S2 (band 0, younger than
// B) waits for B.
static void test_bands_keep_submission_order()
{
    for (int by_slots = 0; by_slots < 2; ++by_slots) {
        Obs obs;
        Fake f0, f1;
        f0.obs = f1.obs = &obs;
        // a 32 x 32 request takes 16384 bytes, an 8 x 8 one 1024
        if (!by_slots)
            f0.cap = f1.cap = 16384 + 512;
        std::mutex gm;
        std::condition_variable gcv;
        bool open = false;
        f0.gate = [&] {
            std::unique_lock<std::mutex> g(gm);
            gcv.wait(g, [&] { return open; });
        };
        Core<Fake> c({&f0, &f1}, band_cfg(by_slots ? 1 : 8));
        c.start();
        Sub s1 = submit_one(c, 8, 8, 1e3, 1);
        while (c.active_count() < 1)
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        Sub b = submit_one(c, 32, 32, 1e3, 2);
        Sub s2 = submit_one(c, 8, 8, 1e3, 3);
        {
            std::lock_guard<std::mutex> g(gm);
            open = true;
        }
        gcv.notify_all();
        for (Sub *s : {&s1, &b, &s2}) {
            la_status rs;
            la_polar_info info;
            std::vector<float> U;
            CHECK(wait_done(c, *s, &rs, &info, &U));
            check_result(*s, rs, info, U);
        }
        const std::vector<uint64_t> order = {s1.id, b.id, s2.id};
        CHECK(obs.admitted == order);
        CHECK(obs.max_live == 1 && !obs.overlap);
        printf("bands_keep_submission_order (%s): ok\n", by_slots ? "slots" : "arena");
    }
}

// A device error in one band fails the other band's requests too.
static void test_bands_device_error()
{
    Obs obs;
    Fake f0, f1;
    f0.obs = f1.obs = &obs;
    f1.fail_tick = 0;
    std::mutex gm;
    std::condition_variable gcv;
    bool open = false;
    f0.gate = [&] {
        std::unique_lock<std::mutex> g(gm);
        gcv.wait(g, [&] { return open; });
    };
    Core<Fake> c({&f0, &f1}, band_cfg(8));
    c.start();
    Sub s = submit_one(c, 12, 12, 1e5, 1);
    while (c.active_count() < 1)
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    Sub b = submit_one(c, 32, 32, 1e3, 2);
    la_status rs;
    la_polar_info info;
    std::vector<float> U;
    CHECK(wait_done(c, b, &rs, &info, &U));
    CHECK(rs == LA_ERR_DEVICE);
    {
        std::lock_guard<std::mutex> g(gm);
        open = true;
    }
    gcv.notify_all();
    CHECK(wait_done(c, s, &rs, &info, &U));
    CHECK(rs == LA_ERR_DEVICE);
    uint64_t id;
    std::vector<float> A(64, 1.0f);
    CHECK(c.submit(8, 8, A.data(), 8, nullptr, &id) == LA_ERR_DEVICE);
    CHECK(c.active_count() == 0 && obs.live == 0);
    const la_serve_stats st = c.stats();
    CHECK(st.failed == 2 && st.completed == 0);
    printf("bands_device_error: ok\n");
}

// The XCD layout of a grouped launch: every tile of every problem exactly
// once, each XCD's share of a problem one contiguous run in tile order,
// fewer than xcds empty entries per problem, and the work (tiles x cost) of
// the XCDs within one tile of the largest cost of each other.
static void test_xcd_layout()
{
    const int X = 8;
    std::vector<std::vector<int64_t>> tiles_cases = {
        {256}, {136}, {3}, {1024, 16, 10, 3, 1}, {7, 7, 7, 7, 7, 7, 7}, {}, {9, 200, 64}};
    std::vector<std::vector<int64_t>> cost_cases = {
        {2048}, {2048}, {128}, {4096, 512, 512, 256, 128}, {64, 64, 64, 64, 64, 64, 64}, {},
        {1024, 2048, 512}};
    for (size_t c = 0; c < tiles_cases.size(); ++c) {
        const auto &tl = tiles_cases[c];
        const auto &co = cost_cases[c];
        const std::vector<Slot> lay = xcd_layout(tl, co, X);
        CHECK(lay.size() % X == 0);
        int64_t total = 0;
        for (int64_t t : tl)
            total += t;
        CHECK((int64_t)lay.size() <= total + (int64_t)(X - 1) * (int64_t)tl.size());
        std::vector<std::vector<int>> seen(tl.size());
        for (size_t p = 0; p < tl.size(); ++p)
            seen[p].assign(tl[p], 0);
        std::vector<double> work(X, 0.0);
        // per XCD and problem: the tiles in list order
        std::vector<std::vector<std::vector<int>>> run(X, std::vector<std::vector<int>>(tl.size()));
        for (size_t i = 0; i < lay.size(); ++i) {
            const Slot s = lay[i];
            if (s.prob < 0)
                continue;
            CHECK(s.prob < (int)tl.size() && s.tile >= 0 && s.tile < tl[s.prob]);
            seen[s.prob][s.tile]++;
            work[i % X] += (double)co[s.prob];
            run[i % X][s.prob].push_back(s.tile);
        }
        for (size_t p = 0; p < tl.size(); ++p)
            for (int v : seen[p])
                CHECK(v == 1);
        for (int x = 0; x < X; ++x)
            for (size_t p = 0; p < tl.size(); ++p)
                for (size_t k = 1; k < run[x][p].size(); ++k)
                    CHECK(run[x][p][k] == run[x][p][k - 1] + 1);
        if (!tl.empty()) {
            const double mx = *std::max_element(work.begin(), work.end());
            const double mn = *std::min_element(work.begin(), work.end());
            CHECK(mx - mn <= (double)*std::max_element(co.begin(), co.end()));
        }
    }
}

int main(int argc, char **argv)
{
    test_mix_and_counts();
    test_arena_slots_and_staging();
    test_queue_full_and_gate();
    test_nonfinite_cap_and_errors();
    test_device_errors();
    test_threads_and_shutdown();
    test_bands_route_and_mix();
    test_bands_tick_independently();
    test_bands_keep_submission_order();
    test_bands_device_error();
    test_xcd_layout();
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("ALL OK\n");
    return 0;
}
