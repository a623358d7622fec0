// Continuous-batching server of polar requests (la_serve_* in la.h): the HIP
// executor of the scheduler in serve_core.h.
//
// Requests are routed by size to one of two bands (square n <= 2048, and
// larger), each with a scheduler thread, a stream of its own (plus side
// streams) and a staging area; the bands tick independently and share the
// arena, the slots and the pinned host buffers.  A band's tick:
//   1. admits its queued requests (FIFO, and no request overtakes an older
//      one of the other band for arena or slots) while a slot is free, the
//      request's device footprint fits the arena (first-fit allocator) and
//      its launch descriptors and tile items fit the band's staging area; for
//      each, the input is copied in, ||A||_F^2 is summed in FP64 and
//      X0 = A / ||A||_F is formed on the device from that sum (Algorithm
//      NS_Polar, first step);
//   2. advances every active request of the band, the new ones included, by
//      one iteration of Algorithm NS_Polar (a preconditioning step, eqs.
//      a_def-RogueMatrix, or a Newton-Schulz step, eq. NewtonSchulz): one
//      grouped Gram launch and one grouped update launch per precision and
//      tile class cover all of them, whatever their sizes; the tick's
//      descriptors, tile items and reduce items go up in one copy, and the
//      launches of a phase run side by side on up to four streams (a launch
//      of a few large-tile problems fills only part of the device);
//   3. reduces the new requests' norms and the Newton-Schulz step norms in one
//      grouped launch and reads them back in one copy: the tick's one wait;
//   4. applies each request's stop test on the host; finished requests get
//      H = (U^T A + A^T U) / 2 (Gram-mode products of U^T A and A^T U in one
//      grouped launch, added in FP64 and written to both triangles), their
//      factors are copied to pinned host buffers and their arena blocks are
//      released.
// A small request thus steps at the pace of its own band and not at that of
// the largest request in flight.
// Every tile of every request is computed by the same kernel code with the
// same tile shape as when the request runs alone, so a request's result is
// bitwise independent of what else is in flight.  Each product accumulates
// over its whole K (square requests up to n = 4096 stay within la_polar's
// FP32 accumulation depth; la_polar_opts.max_acc_k is not used here).
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "la_internal.h"
#include "serve_core.h"

namespace la {
namespace {

constexpr size_t kAlign = 256;
// Staging area of one band; kMaxBands of them at the start of the arena.  A
// staging pass fills its upload region from the start, each launch's
// descriptors followed by its items, then the tick's reduce items, so one copy
// takes them all up; the region is sized as a descriptor budget plus an item
// budget (admission counts both per request).
constexpr size_t kDescBytes = 512u << 10;    // descriptor (and reduce item) budget
constexpr size_t kItemBytes = 3u << 20;      // GroupItem budget
constexpr size_t kUpBytes = kDescBytes + kItemBytes;
constexpr size_t kRedBytes = 512u << 10;     // norms read back
constexpr size_t kBandReserve = kUpBytes + kRedBytes;
constexpr int kMaxSlots = 4096;
// Size bands: square requests up to n = 2048 (m n^2 <= 2048^3) tick apart
// from larger ones.
constexpr int kMaxBands = 2;
constexpr double kBandWork = 2048.0 * 2048.0 * 2048.0;
// launch groups of one staging pass: 3 precisions x 2 tile classes x 2 phases,
// each with its descriptors and its items padded to kAlign
constexpr int kMaxGroups = 12;
static_assert(2 * kMaxSlots * sizeof(double) <= kRedBytes, "norms of one tick");
static_assert(2 * sizeof(ReduceItem) <= sizeof(GemmDesc), "reduce items in a descriptor slot");

size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Pinned host buffers reused across requests (power-of-two size classes), so a
// submit does not pay for a pinned allocation once the pool has warmed up.
class PinnedPool {
  public:
    ~PinnedPool()
    {
        for (void *p : all_)
            (void)hipHostFree(p);   // teardown: nobody to report to
    }
    void *get(size_t bytes, size_t *cls)
    {
        size_t c = 4096;
        while (c < bytes)
            c <<= 1;
        *cls = c;
        std::lock_guard<std::mutex> g(mu_);
        auto &fl = free_[c];
        if (!fl.empty()) {
            void *p = fl.back();
            fl.pop_back();
            return p;
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess)
            return nullptr;
        all_.push_back(p);
        return p;
    }
    void put(void *p, size_t cls)
    {
        if (!p)
            return;
        std::lock_guard<std::mutex> g(mu_);
        free_[cls].push_back(p);
    }

  private:
    std::mutex mu_;
    std::map<size_t, std::vector<void *>> free_;
    std::vector<void *> all_;
};

// Device and host state of one request.
struct DevReq {
    float *A = nullptr, *X[2] = {nullptr, nullptr}, *P = nullptr;
    double *tiles = nullptr, *sumsq = nullptr, *scal = nullptr;
    int cur = 0;
    float *io = nullptr;    // pinned: A on submit, U on completion (m n floats)
    float *hh = nullptr;    // pinned: H (n n floats)
    size_t io_cls = 0, hh_cls = 0;
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

struct Launch {
    int prec, akc, bkc, small;
    std::vector<GemmDesc> probs;
    std::vector<GroupItem> items;
};

// A launch whose descriptors and items are in the staging area.
struct Staged {
    const Launch *L;
    const GemmDesc *dd;
    const GroupItem *di;
};

// Streams beside the executor's own that a phase's launches run on: the
// launches of one phase (one per precision and tile class) are independent,
// and a launch of a few large-tile problems fills only part of the device.
constexpr int kSide = 3;

void add_problem(std::vector<Launch> &ls, int prec, int akc, int bkc, const GemmDesc &d)
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

GemmDesc gram_desc(const float *X1, const float *X2, float *C, int64_t m, int64_t n,
                   float alpha, float gamma, int upper, int prec)
{
    GemmDesc d;
    memset(&d, 0, sizeof d);
    d.A = X1;
    d.lda = n;
    d.B = X2;
    d.ldb = n;
    d.C = C;
    d.ldc = n;
    d.M = n;
    d.N = n;
    d.K = m;
    d.alpha = alpha;
    d.gamma = gamma;
    d.gram = 1;
    d.gram_upper = upper;
    gemm_finalize(d, prec);
    return d;
}

GemmDesc update_desc(const float *X, const float *P, float *Xn, int64_t m, int64_t n, int prec)
{
    GemmDesc d;
    memset(&d, 0, sizeof d);
    d.A = X;
    d.lda = n;
    d.a_kcontig = 1;
    d.B = P;
    d.ldb = n;
    d.C = Xn;
    d.ldc = n;
    d.M = m;
    d.N = n;
    d.K = n;
    gemm_finalize(d, prec);
    return d;
}

// Lays out a launch's items for the per-item grouped kernel (item b runs on
// XCD b % kXcds; serve::xcd_layout); empty items pad the XCD lists.
void xcd_order(Launch &L)
{
    std::vector<int64_t> tiles, cost;
    for (const GemmDesc &d : L.probs) {
        tiles.push_back(d.num_tiles);
        cost.push_back(d.K);
    }
    const std::vector<serve::Slot> lay = serve::xcd_layout(tiles, cost, kXcds);
    L.items.resize(lay.size());
    for (size_t i = 0; i < lay.size(); ++i)
        L.items[i] = GroupItem{lay[i].prob, lay[i].tile};
}

struct HipExec {
    la_context *ctx = nullptr;
    int device = 0;
    char *stage_dev = nullptr;   // this band's staging area (kBandReserve bytes)
    char *req_base = nullptr;    // request state: the arena after every band's staging
    size_t req_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t side[kSide] = {};
    hipEvent_t ev_go = nullptr, ev_side[kSide] = {};
    char *h_stage = nullptr;     // pinned mirror of the staging area
    double *h_red = nullptr;     // pinned: norms read back
    PinnedPool *pool = nullptr;  // shared by the bands

    // ---- the executor interface of serve_core.h
    bool bind() { return hipSetDevice(device) == hipSuccess; }
    size_t capacity() { return req_bytes; }
    size_t footprint(const serve::Req &r)
    {
        const size_t mn = (size_t)r.m * r.n, nn = (size_t)r.n * r.n;
        return up(mn * 4) * 3 + up(nn * 4) + up(max_tiles(r.m, r.n) * 8) +
               up((size_t)sumsq_num_partials() * 8) + up(8 * 8);
    }
    // descriptors and tile items one tick stages for r: a Gram and an update,
    // at the most demanding precision the request may step at (H, staged after
    // the tick's wait, needs no more: two descriptors and twice the Gram's
    // tiles, at most the update's), plus the empty items that pad the XCD
    // lists (fewer than kXcds per problem), plus one descriptor's bytes for
    // its reduce items (its norm when new, its step norm: at most two)
    void stage_need(const serve::Req &r, size_t *descs, size_t *items)
    {
        size_t it = 0;
        int precs[3] = {r.plan.prec_pre, r.plan.prec_ns, r.plan.polish ? (int)PREC_BF16X6 : 0};
        for (int pr : precs) {
            if (!pr)
                continue;
            const GemmDesc g = gram_desc(nullptr, nullptr, nullptr, r.m, r.n, 1.0f, 0.0f, 0, pr);
            const GemmDesc u = update_desc(nullptr, nullptr, nullptr, r.m, r.n, pr);
            it = std::max(it, (size_t)g.num_tiles + (size_t)u.num_tiles);
        }
        const GemmDesc h = gram_desc(nullptr, nullptr, nullptr, r.m, r.n, 1.0f, 0.0f, 1,
                                     r.plan.prec_h);
        *descs = 3;
        *items = std::max(it, 2 * (size_t)h.num_tiles) + 2 * (kXcds - 1);
    }
    // each budget keeps room for the kAlign padding of kMaxGroups launches
    size_t desc_capacity() { return (kDescBytes - kMaxGroups * kAlign) / sizeof(GemmDesc); }
    size_t item_capacity() { return (kItemBytes - kMaxGroups * kAlign) / sizeof(GroupItem); }

    la_status stage_input(serve::Req &r, const float *A, int64_t lda)
    {
        DevReq *d = new (std::nothrow) DevReq;
        if (!d) {
            set_error("la_serve_submit: out of host memory");
            return LA_ERR_OUT_OF_MEMORY;
        }
        const size_t mn = (size_t)r.m * r.n, nn = (size_t)r.n * r.n;
        d->io = (float *)pool->get(mn * 4, &d->io_cls);
        d->hh = (float *)pool->get(nn * 4, &d->hh_cls);
        if (!d->io || !d->hh) {
            pool->put(d->io, d->io_cls);
            pool->put(d->hh, d->hh_cls);
            delete d;
            set_error("la_serve_submit: pinned host allocation failed");
            return LA_ERR_OUT_OF_MEMORY;
        }
        for (int64_t i = 0; i < r.m; ++i)
            memcpy(d->io + i * r.n, A + i * lda, (size_t)r.n * 4);
        r.x = d;
        return LA_OK;
    }
    void drop(serve::Req &r)
    {
        DevReq *d = (DevReq *)r.x;
        if (!d)
            return;
        pool->put(d->io, d->io_cls);
        pool->put(d->hh, d->hh_cls);
        delete d;
        r.x = nullptr;
    }
    void place(serve::Req &r, size_t off)
    {
        DevReq *d = (DevReq *)r.x;
        char *b = req_base + off;
        const size_t mn = (size_t)r.m * r.n, nn = (size_t)r.n * r.n;
        d->A = (float *)b;
        b += up(mn * 4);
        d->X[0] = (float *)b;
        b += up(mn * 4);
        d->X[1] = (float *)b;
        b += up(mn * 4);
        d->P = (float *)b;
        b += up(nn * 4);
        d->tiles = (double *)b;
        b += up(max_tiles(r.m, r.n) * 8);
        d->sumsq = (double *)b;
        b += up((size_t)sumsq_num_partials() * 8);
        d->scal = (double *)b;
        d->cur = 0;
    }
    void retire(serve::Req &) {}

    // streams and events (teardown and failed creation: nothing to report to)
    void release_streams()
    {
        for (int k = 0; k < kSide; ++k) {
            if (ev_side[k])
                (void)hipEventDestroy(ev_side[k]);
            if (side[k])
                (void)hipStreamDestroy(side[k]);
            ev_side[k] = nullptr;
            side[k] = nullptr;
        }
        if (ev_go)
            (void)hipEventDestroy(ev_go);
        if (stream)
            (void)hipStreamDestroy(stream);
        ev_go = nullptr;
        stream = nullptr;
    }
    void copy_out(const serve::Req &r, float *U, float *H)
    {
        const DevReq *d = (const DevReq *)r.x;
        if (U)
            memcpy(U, d->io, (size_t)r.m * r.n * 4);
        if (H)
            memcpy(H, d->hh, (size_t)r.n * r.n * 4);
    }

    // Stage each launch's descriptors, then its items (laid out for the XCDs,
    // xcd_order), in the pinned mirror of the upload region from pos on.
    // Admission keeps a tick's staging within the region; the check here only
    // guards that bound.
    hipError_t stage(std::vector<Launch> &ls, size_t &pos, std::vector<Staged> &out)
    {
        for (auto &L : ls) {
            if (L.items.empty())
                continue;
            xcd_order(L);
            const size_t db = L.probs.size() * sizeof(GemmDesc);
            const size_t ib = L.items.size() * sizeof(GroupItem);
            if (pos + up(db) + ib > kUpBytes)
                return hipErrorOutOfMemory;
            memcpy(h_stage + pos, L.probs.data(), db);
            memcpy(h_stage + pos + up(db), L.items.data(), ib);
            out.push_back(Staged{&L, (const GemmDesc *)(stage_dev + pos),
                                 (const GroupItem *)(stage_dev + pos + up(db))});
            pos += up(db) + up(ib);
        }
        return hipSuccess;
    }

    // One copy for everything staged.
    hipError_t upload(size_t pos)
    {
        return pos ? hipMemcpyAsync(stage_dev, h_stage, pos, hipMemcpyHostToDevice, stream)
                   : hipSuccess;
    }

    // The launches of one phase side by side: the first on the executor's
    // stream, the others on the side streams after everything already queued
    // on it; the executor's stream then waits for all of them.
    hipError_t run_phase(const std::vector<Staged> &st)
    {
        if (st.empty())
            return hipSuccess;
        const int used = std::min<int>((int)st.size() - 1, kSide);
        hipError_t e = hipSuccess;
        if (used > 0)
            e = hipEventRecord(ev_go, stream);
        for (int k = 0; k < used && e == hipSuccess; ++k)
            e = hipStreamWaitEvent(side[k], ev_go, 0);
        for (size_t i = 0; i < st.size() && e == hipSuccess; ++i) {
            const Launch &L = *st[i].L;
            hipStream_t s = i == 0 ? stream : side[(i - 1) % kSide];
            e = launch_gemm_grouped(L.prec, L.akc, L.bkc, L.small, st[i].dd, st[i].di,
                                    (int)L.items.size(), 0, s);
        }
        for (int k = 0; k < used && e == hipSuccess; ++k) {
            e = hipEventRecord(ev_side[k], side[k]);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(stream, ev_side[k], 0);
        }
        return e;
    }

    la_status tick(const std::vector<serve::Req *> &fresh, const std::vector<serve::Req *> &run,
                   std::vector<double> &fro2, std::vector<double> &delta2)
    {
        hipError_t e = hipSuccess;
        // 1. new requests: input, ||A||_F^2 in FP64, X0 = A / ||A||_F on the device
        for (serve::Req *r : fresh) {
            DevReq *d = (DevReq *)r->x;
            if (e == hipSuccess)
                e = hipMemcpyAsync(d->A, d->io, (size_t)r->m * r->n * 4, hipMemcpyHostToDevice,
                                   stream);
            if (e == hipSuccess)
                e = launch_sumsq(d->A, r->m, r->n, r->n, d->sumsq, stream);
            if (e == hipSuccess)
                e = launch_reduce_fixed(d->sumsq, sumsq_num_partials(), d->scal, stream);
            if (e == hipSuccess)
                e = launch_scale_by_norm(d->A, r->n, d->X[0], r->n, r->m, r->n, d->scal, stream);
            d->cur = 0;
        }
        // 2. one step for every running request.  A tick whose requests would
        // fill the device twice over with large tiles runs all of them on large
        // tiles (fewer operand re-reads per flop; the products are the same
        // bits in either tile class); a lighter tick keeps each request's own
        // choice, which favours small tiles for a lone mid-size request.
        int64_t large_load = 0;
        for (serve::Req *r : run) {
            const int pr = r->step_prec();
            large_load += (int64_t)((r->m + tile_m(pr, 0) - 1) / tile_m(pr, 0)) *
                          ((r->n + tile_n(pr, 0) - 1) / tile_n(pr, 0));
        }
        const bool all_large = large_load >= 2 * (int64_t)ctx->num_cus;
        std::vector<Launch> grams, updates;
        std::vector<ReduceItem> red;
        double *dev_d = (double *)(stage_dev + kUpBytes);
        for (serve::Req *r : fresh)
            red.push_back(ReduceItem{((DevReq *)r->x)->scal, 1, dev_d + red.size()});
        for (serve::Req *r : run) {
            DevReq *d = (DevReq *)r->x;
            const PolarPlan &p = r->plan;
            const bool pre = r->precond();
            const int prec = r->step_prec();
            GemmDesc gd = gram_desc(d->X[d->cur], d->X[d->cur], d->P, r->m, r->n,
                                    pre ? (float)(-p.c) : -1.0f, 1.0f, 0, prec);
            GemmDesc ud = update_desc(d->X[d->cur], d->P, d->X[d->cur ^ 1], r->m, r->n, prec);
            if (all_large) {
                gemm_set_class(gd, prec, 0);
                gemm_set_class(ud, prec, 0);
            }
            add_problem(grams, prec, 0, 0, gd);
            if (pre) {
                ud.alpha = (float)p.a;
            } else {
                ud.alpha = 0.5f;
                ud.beta = 1.0f;
                ud.E = d->X[d->cur];
                ud.lde = r->n;
                ud.partials = d->tiles;
                red.push_back(ReduceItem{d->tiles, (int64_t)ud.tiles_m * ud.tiles_n,
                                         dev_d + red.size()});
            }
            add_problem(updates, prec, 1, 0, ud);
        }
        size_t pos = 0;
        std::vector<Staged> sg, su;
        if (e == hipSuccess)
            e = stage(grams, pos, sg);
        if (e == hipSuccess)
            e = stage(updates, pos, su);
        // the reduce items go up with the launches' descriptors and items
        const ReduceItem *dev_ri = (const ReduceItem *)(stage_dev + pos);
        const size_t rb = red.size() * sizeof(ReduceItem);
        if (e == hipSuccess && pos + rb > kUpBytes)
            e = hipErrorOutOfMemory;
        if (e == hipSuccess) {
            memcpy(h_stage + pos, red.data(), rb);
            pos += rb;
            e = upload(pos);
        }
        if (e == hipSuccess)
            e = run_phase(sg);
        if (e == hipSuccess)
            e = run_phase(su);
        // 3. the norms of the new requests and the step norms, one readback
        if (e == hipSuccess && !red.empty()) {
            e = launch_reduce_grouped(dev_ri, (int)red.size(), stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(h_red, dev_d, red.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, stream);
        }
        if (e == hipSuccess)
            e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            set_error("la_serve: device error %s", hipGetErrorString(e));
            return LA_ERR_DEVICE;
        }
        for (size_t i = 0; i < fresh.size(); ++i)
            fro2[i] = h_red[i];
        for (size_t j = fresh.size(); j < red.size(); ++j)
            delta2.push_back(h_red[j]);
        for (serve::Req *r : run)
            ((DevReq *)r->x)->cur ^= 1;
        return LA_OK;
    }

    // H = (U^T A + A^T U) / 2: the upper triangles of U^T A (into the free
    // iterate buffer) and of A^T U (into P) in one grouped Gram-mode launch,
    // then their FP64 sum with the factor 1/2 written to both triangles over A,
    // which is no longer needed; U and H are copied to the pinned buffers.
    la_status finish(const std::vector<serve::Req *> &done)
    {
        std::vector<Launch> hs;
        for (serve::Req *r : done) {
            DevReq *d = (DevReq *)r->x;
            const float *U = d->X[d->cur];
            add_problem(hs, r->plan.prec_h, 0, 0,
                        gram_desc(U, d->A, d->X[d->cur ^ 1], r->m, r->n, 1.0f, 0.0f, 1,
                                  r->plan.prec_h));
            add_problem(hs, r->plan.prec_h, 0, 0,
                        gram_desc(d->A, U, d->P, r->m, r->n, 1.0f, 0.0f, 1, r->plan.prec_h));
        }
        size_t pos = 0;   // the tick's wait has passed: the region is free
        std::vector<Staged> sh;
        hipError_t e = stage(hs, pos, sh);
        if (e == hipSuccess)
            e = upload(pos);
        if (e == hipSuccess)
            e = run_phase(sh);
        for (serve::Req *r : done) {
            if (e != hipSuccess)
                break;
            DevReq *d = (DevReq *)r->x;
            const int64_t stride = d->P - d->X[d->cur ^ 1];   // both in the arena
            e = launch_splitk_sym_reduce(d->X[d->cur ^ 1], stride, 2, r->n, 0.5, 0.0, d->A, r->n,
                                         stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d->io, d->X[d->cur], (size_t)r->m * r->n * 4,
                                   hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d->hh, d->A, (size_t)r->n * r->n * 4, hipMemcpyDeviceToHost,
                                   stream);
        }
        if (e == hipSuccess)
            e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            set_error("la_serve: device error %s", hipGetErrorString(e));
            return LA_ERR_DEVICE;
        }
        return LA_OK;
    }
};

}  // namespace
}  // namespace la

using namespace la;

struct la_server {
    PinnedPool pool;
    HipExec ex[kMaxBands];
    int bands = 0;
    std::unique_ptr<serve::Core<HipExec>> core;

    // streams, events and pinned staging of every band (teardown and failed
    // creation: nothing to report to)
    void release()
    {
        for (HipExec &x : ex) {
            x.release_streams();
            if (x.h_stage)
                (void)hipHostFree(x.h_stage);
            if (x.h_red)
                (void)hipHostFree(x.h_red);
            x.h_stage = nullptr;
            x.h_red = nullptr;
        }
    }
};

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
    constexpr size_t kReserve = kMaxBands * kBandReserve;
    if (arena_bytes < kReserve + (64u << 20)) {
        set_error("la_serve_create: arena of %zu bytes is below the %zu-byte minimum",
                  arena_bytes, kReserve + (64u << 20));
        return LA_ERR_OUT_OF_MEMORY;
    }
    if (cfg && (cfg->bands < 0 || cfg->bands > kMaxBands)) {
        set_error("la_serve_create: bands = %d (0 for the default, 1 or 2)", cfg->bands);
        return LA_ERR_INVALID_ARG;
    }
    std::unique_ptr<la_server> s(new (std::nothrow) la_server);
    if (!s) {
        set_error("la_serve_create: out of host memory");
        return LA_ERR_OUT_OF_MEMORY;
    }
    serve::Config c;
    if (cfg && cfg->max_slots > 0)
        c.max_slots = std::min(cfg->max_slots, kMaxSlots);
    if (cfg && cfg->max_queue > 0)
        c.max_queue = cfg->max_queue;
    s->bands = cfg && cfg->bands > 0 ? cfg->bands : kMaxBands;
    if (s->bands > 1)
        c.band_work.push_back(kBandWork);
    hipError_t e = hipSetDevice(ctx->device);
    std::vector<HipExec *> bands;
    for (int b = 0; b < s->bands && e == hipSuccess; ++b) {
        HipExec &x = s->ex[b];
        x.ctx = ctx;
        x.device = ctx->device;
        x.stage_dev = (char *)arena + b * kBandReserve;
        x.req_base = (char *)arena + kReserve;
        x.req_bytes = (arena_bytes & ~(kAlign - 1)) - kReserve;
        x.pool = &s->pool;
        e = hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking);
        for (int k = 0; k < kSide && e == hipSuccess; ++k)
            e = hipStreamCreateWithFlags(&x.side[k], hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&x.ev_go, hipEventDisableTiming);
        for (int k = 0; k < kSide && e == hipSuccess; ++k)
            e = hipEventCreateWithFlags(&x.ev_side[k], hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&x.h_stage, kBandReserve, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&x.h_red, 2 * kMaxSlots * sizeof(double),
                              hipHostMallocDefault);
        bands.push_back(&x);
    }
    if (e != hipSuccess) {
        // cleanup of a failed create: the first error is the one reported
        s->release();
        set_error("la_serve_create: %s", hipGetErrorString(e));
        return LA_ERR_DEVICE;
    }
    s->core.reset(new (std::nothrow) serve::Core<HipExec>(bands, c));
    if (!s->core) {
        s->release();
        set_error("la_serve_create: out of host memory");
        return LA_ERR_OUT_OF_MEMORY;
    }
    s->core->start();
    *out = s.release();
    return LA_OK;
}

la_status la_serve_submit(la_server *s, int64_t m, int64_t n, const float *A_host, int64_t lda,
                          const la_polar_opts *opts, uint64_t *req_id)
{
    if (!s) {
        set_error("la_serve_submit: NULL server");
        return LA_ERR_INVALID_ARG;
    }
    return s->core->submit(m, n, A_host, lda, opts, req_id);
}

la_status la_serve_poll(la_server *s, uint64_t id, float *U_host, float *H_host,
                        la_polar_info *info, la_status *req_status)
{
    if (!s) {
        set_error("la_serve_poll: NULL server");
        return LA_ERR_INVALID_ARG;
    }
    return s->core->poll(id, U_host, H_host, info, req_status);
}

la_status la_serve_stats_get(la_server *s, la_serve_stats *out)
{
    if (!s || !out) {
        set_error("la_serve_stats_get: NULL argument");
        return LA_ERR_INVALID_ARG;
    }
    *out = s->core->stats();
    out->arena_high_water += kMaxBands * kBandReserve;
    return LA_OK;
}

la_status la_serve_destroy(la_server *s)
{
    if (!s)
        return LA_OK;
    s->core->shutdown();
    // teardown: an error here has no caller to act on it
    for (int b = 0; b < s->bands; ++b)
        (void)hipStreamSynchronize(s->ex[b].stream);
    s->core.reset();
    s->release();
    delete s;
    return LA_OK;
}

}  // extern "C"
