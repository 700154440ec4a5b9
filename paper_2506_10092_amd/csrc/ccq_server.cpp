// Serving loop (include/ccq.h, ccq_server_*): queries arrive from any host
// thread; a dispatcher thread admits them while their workspace fits the
// HBM budget (a device arena allocated once) and a slot is free, and keeps
// the GPU fed: whenever a stream is idle, everything admitted so far goes to
// it as one batched launch (continuous batching), or, with batching off, as
// one ccq_execute per query (the single-launch path).  Completion is seen
// through one event per launch; latency = completion - submission on the
// host's steady clock.
//
// A batched dispatch writes its per-query descriptors (plans, workspace
// regions, outputs, work items) into the stream's descriptor buffer in
// device memory and replays a hipGraph of the launch sequence.  The graph's
// kernel arguments are only that buffer and the arena, so one graph serves
// every dispatch of the same launch shape: the kernel instances with their
// grids and LDS sizes, and the query count rounded up to a power of two.
// Graphs are captured the first time a shape is seen (at most kMaxGraphs
// per stream; the cache is cleared when full).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "ccq_internal.h"

using namespace ccq;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// first-fit allocator over [0, size) with coalescing frees
struct Arena {
    std::map<size_t, size_t> free_;   // offset -> length
    size_t size = 0;
    void init(size_t n) {
        size = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(size_t n, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
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
};

struct Req {
    uint64_t ticket;
    const ccq_plan* plan;
    ccq_result result;
    double t_submit, t_start;
    size_t off, bytes;
};

constexpr size_t kMaxGraphs = 256;

struct Lane {                     // one launch stream
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Req> running;
    unsigned char* desc_host = nullptr;   // pinned staging of the batch descriptor
    unsigned char* desc_dev = nullptr;    // device copy (inside the arena)
    size_t desc_bytes = 0;
    bool busy = false;
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;   // launch shape -> captured sequence
};

void drop_graphs(Lane& L) {
    for (auto& kv : L.graphs) (void)hipGraphExecDestroy(kv.second);
    L.graphs.clear();
}

}  // namespace

struct ccq_server {
    ccq_context* ctx = nullptr;
    ccq_server_config cfg;
    unsigned char* arena_base = nullptr;
    Arena arena;
    std::vector<Lane> lanes;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> incoming;          // submitted, not yet seen by the dispatcher
    std::vector<ccq_completion> done;  // completed, not yet polled
    uint64_t next_ticket = 1;
    int64_t outstanding = 0;           // submitted and not yet completed
    bool stop = false;
    std::atomic<int32_t> fatal{0};     // first HIP error seen by the dispatcher
    std::thread th;

    // dispatcher-only state
    std::deque<Req> pending;           // waiting for budget / a slot
    std::vector<Req> admitted;         // have a workspace region, not yet launched
    int64_t inflight = 0;              // admitted + running
};

namespace {

void complete(ccq_server* s, const Req& r, int32_t status, double t_done) {
    ccq_completion c;
    memset(&c, 0, sizeof c);
    c.ticket = r.ticket;
    c.status = status;
    c.t_submit = r.t_submit;
    c.t_start = r.t_start;
    c.t_done = t_done;
    std::lock_guard<std::mutex> g(s->mu);
    s->done.push_back(c);
    s->outstanding--;
    s->cv.notify_all();
}

// bytes of a batch descriptor for n queries with `items` work items in total
size_t desc_size(size_t n, size_t items) {
    return align256(sizeof(BatchDev)) + 256 + 4 * align256(8 * n + 8) + align256(sizeof(BatchOut) * n + 8) +
           sizeof(BatchItem) * items + 256 * kMaxInstances;
}

int64_t items_of(const ccq_plan* p, int32_t tpi) { return (p->host.n_tiles + tpi - 1) / tpi; }

// Launch what is admitted on `lane` (as many queries as the batch size and
// the descriptor space allow); returns a HIP error or hipSuccess.
hipError_t launch_lane(ccq_server* s, Lane& L) {
    std::vector<Req> reqs;
    const int32_t tpi0 = s->cfg.tiles_per_item > 0 ? s->cfg.tiles_per_item : 64;
    size_t take = 0, items = 0;
    while (take < s->admitted.size() && (int)take < std::max(1, s->cfg.max_batch)) {
        const size_t more = (size_t)items_of(s->admitted[take].plan, tpi0);
        if (take > 0 && desc_size(take + 1, items + more) > L.desc_bytes) break;
        items += more;
        ++take;
    }
    reqs.assign(s->admitted.begin(), s->admitted.begin() + take);
    s->admitted.erase(s->admitted.begin(), s->admitted.begin() + take);
    // work-item size for this dispatch: small enough that the dispatch's
    // tiles make about four items per compute unit (a lone small query then
    // spreads over the GPU as a single launch would), at most tiles_per_item,
    // and large enough for the descriptor buffer
    int64_t all_tiles = 0;
    for (auto& r : reqs) all_tiles += r.plan->host.n_tiles;
    int32_t tpi_d = (int32_t)std::max<int64_t>(1, std::min<int64_t>(tpi0, (all_tiles + 4 * s->ctx->cus - 1) /
                                                                         std::max(1, 4 * s->ctx->cus)));
    for (;;) {
        size_t it = 0;
        for (auto& r : reqs) it += (size_t)items_of(r.plan, tpi_d);
        if (tpi_d >= tpi0 || desc_size(reqs.size(), it) <= L.desc_bytes) break;
        tpi_d = std::min<int32_t>(tpi0, tpi_d * 2);
    }
    const double t = now_s();
    for (auto& r : reqs) r.t_start = t;
    hipError_t e = hipSuccess;
    // A dispatch of one query gains nothing from a batch: its own
    // single-query kernels spread it over the whole GPU at once.
    if (!s->cfg.batching || reqs.size() == 1) {
        for (auto& r : reqs) {
            e = launch_query(r.plan->host, r.plan->dev, s->arena_base + r.off, L.stream, r.result.keys,
                             r.result.counts, r.result.aggs, r.result.n_groups, r.result.status, r.plan->grid_fused,
                             nullptr, nullptr);
            if (e != hipSuccess) break;
        }
    } else {
        // descriptor: BatchDev | counters | plans | regions | clear sizes | outs | items per group
        const int n = (int)reqs.size();
        const int32_t tpi = tpi_d;
        int group_of[3][kVariants];
        for (auto& row : group_of)
            for (int& g : row) g = -1;
        int n_groups = 0;
        std::vector<std::vector<BatchItem>> items;
        std::vector<int> glds, ggrid, gk, gw, gb;
        std::vector<const DevPlan*> plans_host(n), plans_dev(n);
        std::vector<int64_t> region(n), clear(n);
        std::vector<BatchOut> outs(n);
        std::vector<int32_t> big;
        for (int i = 0; i < n; ++i) {
            const DevPlan& p = reqs[i].plan->host;
            const int ki = p.kmax <= 2 ? 0 : p.kmax <= 4 ? 1 : 2, wi = variant_of(kernel_w0(p), p.fast_big, p.lds_dyn_bytes);
            int& g = group_of[ki][wi];
            if (g < 0) {
                g = n_groups++;
                items.emplace_back();
                glds.push_back(0);
                gk.push_back(p.kmax);
                gw.push_back(kernel_w0(p));
                gb.push_back(p.fast_big);
            }
            glds[g] = std::max(glds[g], p.lds_dyn_bytes);
            for (int64_t t0 = 0; t0 < p.n_tiles; t0 += tpi) {
                BatchItem it;
                it.query = i;
                it.first_tile = t0;
                it.n_tiles = (int32_t)std::min<int64_t>(tpi, p.n_tiles - t0);
                items[g].push_back(it);
            }
            plans_host[i] = &reqs[i].plan->host;
            plans_dev[i] = reqs[i].plan->dev;
            region[i] = (int64_t)reqs[i].off;
            clear[i] = (int64_t)reqs[i].plan->ws.total;
            outs[i] = BatchOut{reqs[i].result.keys, reqs[i].result.counts, reqs[i].result.aggs,
                               reqs[i].result.n_groups, reqs[i].result.status};
            if (p.n_keys > 0 && p.n_groups > kBatchFinMaxGroups) big.push_back(i);
        }
        for (int g = 0; g < n_groups; ++g) ggrid.push_back(batch_grid_limit(gk[g], gw[g], gb[g], glds[g], s->ctx->cus));
        size_t off = align256(sizeof(BatchDev));
        const size_t o_cnt = off;
        off = align256(off + sizeof(int32_t) * kMaxInstances);
        const size_t o_plans = off;
        off = align256(off + sizeof(void*) * n);
        const size_t o_region = off;
        off = align256(off + sizeof(int64_t) * n);
        const size_t o_clear = off;
        off = align256(off + sizeof(int64_t) * n);
        const size_t o_outs = off;
        off = align256(off + sizeof(BatchOut) * n);
        std::vector<size_t> o_items(n_groups);
        for (int g = 0; g < n_groups; ++g) {
            o_items[g] = off;
            off = align256(off + sizeof(BatchItem) * std::max<size_t>(1, items[g].size()));
        }
        if (off > L.desc_bytes) return hipErrorOutOfMemory;   // the caller keeps batches small enough
        unsigned char* h = L.desc_host;
        unsigned char* d = L.desc_dev;
        BatchDev H;
        memset(&H, 0, sizeof H);
        H.plans = (const DevPlan* const*)(d + o_plans);
        H.region = (const int64_t*)(d + o_region);
        H.region_clear = (const int64_t*)(d + o_clear);
        H.outs = (const BatchOut*)(d + o_outs);
        H.counters = (int32_t*)(d + o_cnt);
        H.n = n;
        H.n_groups_used = n_groups;
        for (int g = 0; g < n_groups; ++g) {
            H.groups[g].items = (const BatchItem*)(d + o_items[g]);
            H.groups[g].n_items = (int32_t)items[g].size();
            H.groups[g].kmax = gk[g];
            H.groups[g].w0 = gw[g];
            H.groups[g].big = gb[g];
        }
        memcpy(h, &H, sizeof H);
        memcpy(h + o_plans, plans_dev.data(), sizeof(void*) * n);
        memcpy(h + o_region, region.data(), sizeof(int64_t) * n);
        memcpy(h + o_clear, clear.data(), sizeof(int64_t) * n);
        memcpy(h + o_outs, outs.data(), sizeof(BatchOut) * n);
        for (int g = 0; g < n_groups; ++g)
            if (!items[g].empty()) memcpy(h + o_items[g], items[g].data(), sizeof(BatchItem) * items[g].size());
        e = hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, L.stream);
        if (e == hipSuccess && !s->cfg.no_graphs && big.empty()) {
            // the launch shape: query count rounded up to a power of two, then
            // each group's kernel instance, grid and LDS
            int32_t nb = 1;
            while (nb < n) nb <<= 1;
            std::vector<int64_t> key = {nb, n_groups};
            for (int g = 0; g < n_groups; ++g) key.insert(key.end(), {gk[g], gw[g], gb[g], ggrid[g], glds[g]});
            auto it = L.graphs.find(key);
            if (it == L.graphs.end()) {
                if (L.graphs.size() >= kMaxGraphs) drop_graphs(L);
                hipGraph_t graph = nullptr;
                hipGraphExec_t exec = nullptr;
                e = hipStreamBeginCapture(L.stream, hipStreamCaptureModeRelaxed);
                if (e == hipSuccess) {
                    const hipError_t le = launch_batch(H, (const BatchDev*)d, plans_host.data(), plans_dev.data(),
                                                       region.data(), outs.data(), s->arena_base, ggrid.data(),
                                                       glds.data(), nullptr, 0, L.stream, nullptr, nullptr, nb);
                    e = hipStreamEndCapture(L.stream, &graph);
                    if (le != hipSuccess) e = le;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                if (graph) (void)hipGraphDestroy(graph);
                if (e == hipSuccess) it = L.graphs.emplace(key, exec).first;
            }
            if (e == hipSuccess) e = hipGraphLaunch(it->second, L.stream);
        } else if (e == hipSuccess) {
            e = launch_batch(H, (const BatchDev*)d, plans_host.data(), plans_dev.data(), region.data(), outs.data(),
                             s->arena_base, ggrid.data(), glds.data(), big.data(), (int32_t)big.size(), L.stream);
        }
    }
    if (e == hipSuccess) e = hipEventRecord(L.done, L.stream);
    L.running = std::move(reqs);
    L.busy = true;
    return e;
}

void dispatcher(ccq_server* s) {
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        bool idle_wait = true;
        {
            std::unique_lock<std::mutex> g(s->mu);
            if (s->stop && s->incoming.empty() && s->outstanding == 0) return;
            while (!s->incoming.empty()) {
                s->pending.push_back(s->incoming.front());
                s->incoming.pop_front();
            }
        }
        // completions
        for (Lane& L : s->lanes) {
            if (!L.busy) continue;
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) continue;
            const double t = now_s();
            const int32_t st = q == hipSuccess ? CCQ_OK : CCQ_E_HIP;
            if (q != hipSuccess) s->fatal.store((int32_t)q);
            for (const Req& r : L.running) {
                s->arena.release(r.off, r.bytes);
                s->inflight--;
                complete(s, r, st, t);
            }
            L.running.clear();
            L.busy = false;
            idle_wait = false;
        }
        // admission by budget and slots
        while (!s->pending.empty() && s->inflight < s->cfg.max_inflight) {
            Req& r = s->pending.front();
            r.bytes = align256(std::max<size_t>(r.plan->ws.total, 256));
            if (r.bytes > s->arena.size) {
                Req dead = r;
                s->pending.pop_front();
                dead.t_start = now_s();   // never launched: start = done = rejection time
                complete(s, dead, CCQ_E_BUDGET, dead.t_start);
                continue;
            }
            size_t off;
            if (!s->arena.alloc(r.bytes, &off)) break;      // wait for frees
            r.off = off;
            s->admitted.push_back(r);
            s->pending.pop_front();
            s->inflight++;
        }
        // launch on idle streams
        for (Lane& L : s->lanes) {
            if (s->admitted.empty()) break;
            if (L.busy) continue;
            const hipError_t e = launch_lane(s, L);
            idle_wait = false;
            if (e != hipSuccess) {
                s->fatal.store((int32_t)e);
                (void)hipStreamSynchronize(L.stream);
                for (const Req& r : L.running) {
                    s->arena.release(r.off, r.bytes);
                    s->inflight--;
                    complete(s, r, CCQ_E_HIP, now_s());
                }
                L.running.clear();
                L.busy = false;
            }
        }
        if (idle_wait) {
            bool any_busy = false;
            for (Lane& L : s->lanes) any_busy = any_busy || L.busy;
            std::unique_lock<std::mutex> g(s->mu);
            if (any_busy)
                s->cv.wait_for(g, std::chrono::microseconds(20));
            else if (s->incoming.empty() && !s->stop)
                s->cv.wait_for(g, std::chrono::milliseconds(2));
        }
    }
}

}  // namespace

extern "C" {

double ccq_now(void) { return now_s(); }

ccq_status ccq_server_create(ccq_context* ctx, const ccq_server_config* cfg, ccq_server** out) {
    if (!out) return fail(CCQ_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!cfg || cfg->hbm_budget_bytes < 4096 || cfg->max_inflight < 1)
        return fail(CCQ_E_INVALID, "config needs hbm_budget_bytes >= 4096 and max_inflight >= 1");
    if (cfg->tiles_per_item < 0 || cfg->tiles_per_item > kMaxTilesPerItem)
        return fail(CCQ_E_INVALID, "tiles_per_item must be in 0..%d", (int)kMaxTilesPerItem);
    if (!ctx || ctx->device < 0) return fail(CCQ_E_INVALID, "server needs a device context");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    ccq_server* s = new (std::nothrow) ccq_server;
    if (!s) return fail(CCQ_E_NOMEM, "out of host memory");
    s->ctx = ctx;
    s->cfg = *cfg;
    if (s->cfg.max_batch <= 0) s->cfg.max_batch = s->cfg.max_inflight;
    if (s->cfg.n_streams <= 0) s->cfg.n_streams = 2;
    // launch descriptor space per stream, carved from the budget
    const size_t desc_bytes = align256(std::max<size_t>(desc_size((size_t)s->cfg.max_batch, 0) * 2, 16u << 20));
    const size_t total = (size_t)cfg->hbm_budget_bytes;
    if (desc_bytes * s->cfg.n_streams >= total) {
        delete s;
        return fail(CCQ_E_BUDGET, "budget too small for the launch descriptors");
    }
    e = hipMalloc(&s->arena_base, total);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "hipMalloc(server arena)");
    }
    s->arena.init(total - desc_bytes * s->cfg.n_streams);
    for (int i = 0; i < s->cfg.n_streams; ++i) {
        Lane L;
        e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void**)&L.desc_host, desc_bytes, hipHostMallocDefault);
        L.desc_dev = s->arena_base + s->arena.size + desc_bytes * i;
        L.desc_bytes = desc_bytes;
        s->lanes.push_back(L);
        if (e != hipSuccess) {
            ccq_server_destroy(s);
            return hip_fail(e, "server streams");
        }
    }
    s->th = std::thread(dispatcher, s);
    *out = s;
    return ok();
}

ccq_status ccq_server_submit(ccq_server* s, const ccq_plan* p, const ccq_result* r, uint64_t* ticket) {
    if (!s || !p || !r) return fail(CCQ_E_INVALID, "server, plan or result is NULL");
    if (p->ctx->device != s->ctx->device) return fail(CCQ_E_INVALID, "plan is on another device");
    if (r->capacity < p->max_groups) return fail(CCQ_E_CAPACITY, "result capacity below the plan's max groups");
    if (s->fatal.load()) return fail(CCQ_E_HIP, "server stopped after a HIP error (%d)", (int)s->fatal.load());
    const int32_t tpi = s->cfg.tiles_per_item > 0 ? s->cfg.tiles_per_item : 64;
    if (desc_size(1, (size_t)items_of(p, tpi)) > s->lanes[0].desc_bytes)
        return fail(CCQ_E_UNSUPPORTED, "query has too many work items for the server's launch descriptors");
    Req q;
    memset(&q, 0, sizeof q);
    q.plan = p;
    q.result = *r;
    q.t_submit = now_s();
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(CCQ_E_BUSY, "server is stopping");
    q.ticket = s->next_ticket++;
    s->incoming.push_back(q);
    s->outstanding++;
    s->cv.notify_all();
    if (ticket) *ticket = q.ticket;
    return ok();
}

ccq_status ccq_server_poll(ccq_server* s, ccq_completion* out, int32_t max, int32_t* n) {
    if (!s || !n || (max > 0 && !out)) return fail(CCQ_E_INVALID, "bad poll arguments");
    std::lock_guard<std::mutex> g(s->mu);
    const int32_t k = (int32_t)std::min<size_t>(s->done.size(), (size_t)std::max(max, 0));
    for (int32_t i = 0; i < k; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n = k;
    return ok();
}

ccq_status ccq_server_drain(ccq_server* s, double timeout_s) {
    if (!s) return fail(CCQ_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> g(s->mu);
    const bool ok_ = s->cv.wait_for(g, std::chrono::duration<double>(timeout_s), [&] { return s->outstanding == 0; });
    if (!ok_) return fail(CCQ_E_BUSY, "queries still outstanding after %.3f s", timeout_s);
    return ok();
}

void ccq_server_destroy(ccq_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(s->ctx->device);
    for (Lane& L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.desc_host) (void)hipHostFree(L.desc_host);
        drop_graphs(L);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
}

}  // extern "C"
