// Batched execution (include/ccq.h, ccq_batch_*): many compiled plans run as
// one launch sequence -- a clear, one persistent launch per kernel instance
// whose workgroups pull (query, tile range) work items from a device counter,
// and a finalize with one workgroup per query -- optionally captured once as
// a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "ccq_internal.h"

using namespace ccq;

struct ccq_batch {
    ccq_context* ctx = nullptr;
    std::vector<const ccq_plan*> plans;
    std::vector<ccq_result> results;
    int32_t tiles_per_item = 0;
    int32_t use_graph = 0;

    // layout
    std::vector<int64_t> region;     // byte offset of each query's region in the workspace
    size_t ws_total = 0;
    std::vector<int32_t> big;        // queries finalized by the multi-block kernels

    // per kernel instance
    int n_groups_used = 0;
    int group_of[3][kVariants];      // [kmax index][variant] -> group or -1
    std::vector<int> group_lds, group_grid;
    std::vector<std::vector<BatchItem>> group_items;
    int64_t n_items = 0;

    // device descriptors
    void* dblob = nullptr;
    BatchDev host;
    std::vector<const DevPlan*> plans_host, plans_dev;
    std::vector<BatchOut> outs;

    // cached graph for (workspace, stream)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    void* g_ws = nullptr;
    hipStream_t g_stream = nullptr;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int kidx(int kmax) { return kmax <= 2 ? 0 : kmax <= 4 ? 1 : 2; }

// FNV-1a over the words that decide a batch's launch shapes
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(uint64_t x) {
        for (int i = 0; i < 8; ++i) {
            h ^= (x >> (8 * i)) & 0xFF;
            h *= 1099511628211ull;
        }
    }
};

// The tuning cache's key of a batch: the device (architecture, CUs), the
// candidate list, and per query its kernel instance, nominal tiles, groups,
// accumulators and LDS bytes.
uint64_t tune_key(const ccq_batch* b, const int32_t* cand, int32_t n_cand) {
    Fnv f;
    for (char c : b->ctx->arch) f.add((uint64_t)(unsigned char)c);
    f.add((uint64_t)b->ctx->cus);
    f.add((uint64_t)n_cand);
    for (int i = 0; i < n_cand; ++i) f.add((uint64_t)(uint32_t)cand[i]);
    f.add((uint64_t)b->plans.size());
    for (const ccq_plan* p : b->plans) {
        const DevPlan& d = p->host;
        f.add((uint64_t)(uint32_t)d.kmax);
        f.add((uint64_t)(int64_t)kernel_w0(d));
        f.add((uint64_t)(uint32_t)d.fast_big);
        f.add((uint64_t)d.n_tiles);
        f.add((uint64_t)d.n_groups);
        f.add((uint64_t)(uint32_t)d.n_sums);
        f.add((uint64_t)(uint32_t)d.lds_dyn_bytes);
    }
    return f.h;
}

int widx(const DevPlan& p) { return variant_of(kernel_w0(p), p.fast_big, p.lds_dyn_bytes); }

void drop_graph(ccq_batch* b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->g_ws = nullptr;
    b->g_stream = nullptr;
}

// (Re)build work items and the device descriptor blob.
ccq_status build_items(ccq_batch* b) {
    drop_graph(b);
    const int n = (int)b->plans.size();
    const int32_t tpi = std::max<int32_t>(1, b->tiles_per_item);
    for (auto& v : b->group_items) v.clear();
    // biggest queries first, so the last items taken are small
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->plans[x]->host.n_tiles > b->plans[y]->host.n_tiles; });
    b->n_items = 0;
    for (int q : order) {
        const DevPlan& p = b->plans[q]->host;
        const int g = b->group_of[kidx(p.kmax)][widx(p)];
        for (int64_t t = 0; t < p.n_tiles; t += tpi) {
            BatchItem it;
            it.query = q;
            it.first_tile = t;
            it.n_tiles = (int32_t)std::min<int64_t>(tpi, p.n_tiles - t);
            b->group_items[g].push_back(it);
            ++b->n_items;
        }
    }
    // blob: BatchDev | counters | plan pointers | regions | clear sizes | outs | items of each group
    size_t off = align256(sizeof(BatchDev));
    const size_t off_counters = off;
    off = align256(off + sizeof(int32_t) * kMaxInstances);
    const size_t off_plans = off;
    off = align256(off + sizeof(void*) * n);
    const size_t off_region = off;
    off = align256(off + sizeof(int64_t) * n);
    const size_t off_clear = off;
    off = align256(off + sizeof(int64_t) * n);
    const size_t off_outs = off;
    off = align256(off + sizeof(BatchOut) * n);
    std::vector<size_t> off_items(b->n_groups_used);
    for (int g = 0; g < b->n_groups_used; ++g) {
        off_items[g] = off;
        off = align256(off + sizeof(BatchItem) * std::max<size_t>(1, b->group_items[g].size()));
    }
    std::vector<unsigned char> blob(off, 0);
    if (b->dblob) (void)hipFree(b->dblob);
    b->dblob = nullptr;
    hipError_t e = hipMalloc(&b->dblob, blob.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(batch)");
    unsigned char* d = (unsigned char*)b->dblob;
    BatchDev& H = b->host;
    memset(&H, 0, sizeof H);
    H.plans = (const DevPlan* const*)(d + off_plans);
    H.region = (const int64_t*)(d + off_region);
    H.region_clear = (const int64_t*)(d + off_clear);
    H.counters = (int32_t*)(d + off_counters);
    H.outs = (const BatchOut*)(d + off_outs);
    H.n = n;
    H.n_groups_used = b->n_groups_used;
    for (int g = 0; g < b->n_groups_used; ++g) {
        H.groups[g].items = (const BatchItem*)(d + off_items[g]);
        H.groups[g].n_items = (int32_t)b->group_items[g].size();
    }
    for (int ki = 0; ki < 3; ++ki)
        for (int wi = 0; wi < kVariants; ++wi) {
            const int g = b->group_of[ki][wi];
            if (g < 0) continue;
            H.groups[g].kmax = ki == 0 ? 2 : ki == 1 ? 4 : 8;
            H.groups[g].w0 = variant_w0(wi);
            H.groups[g].big = variant_big(wi);
        }
    memcpy(blob.data(), &H, sizeof H);
    memcpy(blob.data() + off_plans, b->plans_dev.data(), sizeof(void*) * n);
    memcpy(blob.data() + off_region, b->region.data(), sizeof(int64_t) * n);
    std::vector<int64_t> clear(n);
    for (int i = 0; i < n; ++i) clear[i] = (int64_t)b->plans[i]->ws.total;
    memcpy(blob.data() + off_clear, clear.data(), sizeof(int64_t) * n);
    memcpy(blob.data() + off_outs, b->outs.data(), sizeof(BatchOut) * n);
    for (int g = 0; g < b->n_groups_used; ++g)
        if (!b->group_items[g].empty())
            memcpy(blob.data() + off_items[g], b->group_items[g].data(), sizeof(BatchItem) * b->group_items[g].size());
    e = hipMemcpy(b->dblob, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(batch)");
    return CCQ_OK;
}

ccq_status launch(ccq_batch* b, unsigned char* ws, hipStream_t s, hipEvent_t ev0 = nullptr,
                  hipEvent_t ev1 = nullptr) {
    hipError_t e = launch_batch(b->host, (const BatchDev*)b->dblob, b->plans_host.data(), b->plans_dev.data(),
                                b->region.data(), b->outs.data(), ws, b->group_grid.data(), b->group_lds.data(),
                                b->big.data(), (int32_t)b->big.size(), s, ev0, ev1);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return CCQ_OK;
}

}  // namespace

extern "C" {

ccq_status ccq_batch_create(ccq_context* ctx, const ccq_plan* const* plans, int32_t n, const ccq_result* results,
                            const ccq_batch_opts* opts, ccq_batch** out) {
    if (!out) return fail(CCQ_E_INVALID, "out is NULL");
    *out = nullptr;
    if (opts && (opts->tiles_per_item < 0 || opts->tiles_per_item > kMaxTilesPerItem))
        return fail(CCQ_E_INVALID, "tiles_per_item must be in 0..%d", (int)kMaxTilesPerItem);
    if (!ctx || ctx->device < 0) return fail(CCQ_E_INVALID, "batch needs a device context");
    if (n < 0 || (n > 0 && (!plans || !results))) return fail(CCQ_E_INVALID, "bad plan / result arrays");
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return fail(CCQ_E_INVALID, "plan %d is NULL", i);
        if (plans[i]->ctx->device != ctx->device) return fail(CCQ_E_INVALID, "plan %d is on another device", i);
        const ccq_result& r = results[i];
        if (r.capacity < plans[i]->max_groups)
            return fail(CCQ_E_CAPACITY, "result %d: capacity %lld < max groups %lld", i, (long long)r.capacity,
                        (long long)plans[i]->max_groups);
        if (!r.counts || !r.n_groups || !r.status || (plans[i]->host.n_keys && !r.keys) ||
            (plans[i]->host.n_aggs && !r.aggs))
            return fail(CCQ_E_INVALID, "result %d: buffers missing", i);
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    ccq_batch* b = new (std::nothrow) ccq_batch;
    if (!b) return fail(CCQ_E_NOMEM, "out of host memory");
    b->ctx = ctx;
    b->plans.assign(plans, plans + n);
    b->results.assign(results, results + n);
    b->tiles_per_item = opts && opts->tiles_per_item > 0 ? opts->tiles_per_item : 64;
    b->use_graph = opts ? opts->use_graph : 0;
    for (auto& row : b->group_of)
        for (int& g : row) g = -1;
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const DevPlan& p = plans[i]->host;
        b->region.push_back((int64_t)off);
        off = align256(off + plans[i]->ws.total);
        int& g = b->group_of[kidx(p.kmax)][widx(p)];
        if (g < 0) {
            g = b->n_groups_used++;
            b->group_lds.push_back(0);
            b->group_items.emplace_back();
        }
        b->group_lds[g] = std::max(b->group_lds[g], p.lds_dyn_bytes);
        if (p.n_keys > 0 && p.n_groups > kBatchFinMaxGroups) b->big.push_back(i);
        b->plans_host.push_back(&plans[i]->host);
        b->plans_dev.push_back(plans[i]->dev);
        BatchOut o;
        o.keys = results[i].keys;
        o.counts = results[i].counts;
        o.aggs = results[i].aggs;
        o.n_groups = results[i].n_groups;
        o.status = results[i].status;
        b->outs.push_back(o);
    }
    b->ws_total = std::max<size_t>(off, 256);
    b->group_grid.resize(b->n_groups_used);
    for (int ki = 0; ki < 3; ++ki)
        for (int wi = 0; wi < kVariants; ++wi) {
            const int g = b->group_of[ki][wi];
            if (g < 0) continue;
            b->group_grid[g] = batch_grid_limit(ki == 0 ? 2 : ki == 1 ? 4 : 8, variant_w0(wi), variant_big(wi),
                                                b->group_lds[g], ctx->cus);
        }
    if (ccq_status s = build_items(b)) {
        ccq_batch_destroy(b);
        return s;
    }
    *out = b;
    return ok();
}

void ccq_batch_destroy(ccq_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    drop_graph(b);
    if (b->dblob) (void)hipFree(b->dblob);
    delete b;
}

ccq_status ccq_batch_info(const ccq_batch* b, size_t* workspace_bytes, int64_t* n_items) {
    if (!b) return fail(CCQ_E_INVALID, "batch is NULL");
    if (workspace_bytes) *workspace_bytes = b->ws_total;
    if (n_items) *n_items = b->n_items;
    return ok();
}

ccq_status ccq_batch_set_tiles_per_item(ccq_batch* b, int32_t tiles_per_item) {
    if (!b) return fail(CCQ_E_INVALID, "batch is NULL");
    if (tiles_per_item < 1 || tiles_per_item > kMaxTilesPerItem)
        return fail(CCQ_E_INVALID, "tiles_per_item must be in 1..%d", (int)kMaxTilesPerItem);
    hipError_t e = hipSetDevice(b->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    b->tiles_per_item = tiles_per_item;
    if (ccq_status s = build_items(b)) return s;
    return ok();
}

ccq_status ccq_batch_execute(ccq_batch* b, void* workspace, size_t workspace_bytes, void* stream) {
    return ccq_batch_execute_ex(b, workspace, workspace_bytes, stream, nullptr);
}

ccq_status ccq_batch_execute_ex(ccq_batch* b, void* workspace, size_t workspace_bytes, void* stream,
                                const ccq_exec_opts* opts) {
    if (!b) return fail(CCQ_E_INVALID, "batch is NULL");
    if (!workspace || ((uintptr_t)workspace & 255)) return fail(CCQ_E_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes < b->ws_total)
        return fail(CCQ_E_CAPACITY, "workspace of %zu bytes, batch needs %zu", workspace_bytes, b->ws_total);
    hipError_t e = hipSetDevice(b->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    unsigned char* ws = (unsigned char*)workspace;
    const bool timed = opts && (opts->fused_begin || opts->fused_end);
    if (!b->use_graph || s == nullptr || timed) {
        if (ccq_status st = launch(b, ws, s, opts ? (hipEvent_t)opts->fused_begin : nullptr,
                                   opts ? (hipEvent_t)opts->fused_end : nullptr))
            return st;
        return ok();
    }
    if (!b->gexec || b->g_ws != workspace || b->g_stream != s) {
        drop_graph(b);
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        ccq_status st = launch(b, ws, s);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        b->graph = g;
        e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return hip_fail(e, "hipGraphInstantiate");
        }
        b->g_ws = workspace;
        b->g_stream = s;
    }
    e = hipGraphLaunch(b->gexec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return ok();
}

ccq_status ccq_batch_autotune(ccq_batch* b, void* workspace, size_t workspace_bytes, void* stream,
                              const int32_t* candidates, int32_t n_candidates, int32_t reps, int32_t* best,
                              float* best_ms) {
    if (!b || !candidates || n_candidates < 1 || reps < 1) return fail(CCQ_E_INVALID, "bad autotune arguments");
    // the context's tuning cache first
    const uint64_t key = tune_key(b, candidates, n_candidates);
    {
        std::lock_guard<std::mutex> g(b->ctx->tune_mu);
        auto it = b->ctx->tune.find(key);
        if (it != b->ctx->tune.end() &&
            std::find(candidates, candidates + n_candidates, it->second.first) != candidates + n_candidates) {
            if (ccq_status st = ccq_batch_set_tiles_per_item(b, it->second.first)) return st;
            if (best) *best = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            return ok();
        }
    }
    hipError_t e = hipSetDevice(b->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    int32_t arg_best = candidates[0];
    float t_best = 3.0e38f;
    ccq_status st = CCQ_OK;
    for (int c = 0; c < n_candidates && st == CCQ_OK; ++c) {
        if ((st = ccq_batch_set_tiles_per_item(b, candidates[c]))) break;
        if ((st = ccq_batch_execute(b, workspace, workspace_bytes, stream))) break;   // warm
        std::vector<float> t;
        for (int r = 0; r < reps && st == CCQ_OK; ++r) {
            (void)hipEventRecord(e0, s);
            st = ccq_batch_execute(b, workspace, workspace_bytes, stream);
            (void)hipEventRecord(e1, s);
            if ((e = hipEventSynchronize(e1)) != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t.push_back(ms);
        }
        if (st) break;
        std::sort(t.begin(), t.end());
        const float med = t[t.size() / 2];
        if (med < t_best) {
            t_best = med;
            arg_best = candidates[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    if ((st = ccq_batch_set_tiles_per_item(b, arg_best))) return st;
    {
        std::lock_guard<std::mutex> g(b->ctx->tune_mu);
        b->ctx->tune[key] = {arg_best, t_best};
    }
    if (best) *best = arg_best;
    if (best_ms) *best_ms = t_best;
    return ok();
}

static const char kTuneHeader[] = "ccq-tune-cache 1";

ccq_status ccq_tune_cache_load(ccq_context* ctx, const char* path, int64_t* n_entries) {
    if (n_entries) *n_entries = 0;
    if (!ctx || !path) return fail(CCQ_E_INVALID, "context or path is NULL");
    FILE* f = fopen(path, "r");
    if (!f) {
        if (errno == ENOENT) return ok();        // no cache yet
        return fail(CCQ_E_INVALID, "cannot open %s: %s", path, strerror(errno));
    }
    char line[256];
    std::vector<std::pair<uint64_t, std::pair<int32_t, float>>> got;
    bool header = false, bad = false;
    while (fgets(line, sizeof line, f)) {
        if (!header) {
            header = strncmp(line, kTuneHeader, sizeof kTuneHeader - 1) == 0;
            if (!header) bad = true;
            if (bad) break;
            continue;
        }
        uint64_t key = 0;
        int32_t tpi = 0;
        float ms = 0;
        char extra = 0;
        const int n = sscanf(line, "%" SCNx64 " %" SCNd32 " %f %c", &key, &tpi, &ms, &extra);
        if (n != 3 || tpi < 1 || tpi > kMaxTilesPerItem || !(ms >= 0)) {
            bad = true;
            break;
        }
        got.push_back({key, {tpi, ms}});
    }
    fclose(f);
    if (bad || !header) return fail(CCQ_E_INVALID, "%s is not a tuning cache (line: %.60s)", path, line);
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    for (const auto& x : got) ctx->tune[x.first] = x.second;
    if (n_entries) *n_entries = (int64_t)got.size();
    return ok();
}

ccq_status ccq_tune_cache_save(ccq_context* ctx, const char* path, int64_t* n_entries) {
    if (n_entries) *n_entries = 0;
    if (!ctx || !path) return fail(CCQ_E_INVALID, "context or path is NULL");
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return fail(CCQ_E_INVALID, "cannot write %s: %s", tmp.c_str(), strerror(errno));
    int64_t n = 0;
    bool okw = fprintf(f, "%s\n", kTuneHeader) > 0;
    {
        std::lock_guard<std::mutex> g(ctx->tune_mu);
        for (const auto& x : ctx->tune) {
            okw = okw && fprintf(f, "%016" PRIx64 " %" PRId32 " %.6g\n", x.first, x.second.first, x.second.second) > 0;
            ++n;
        }
    }
    okw = (fclose(f) == 0) && okw;
    if (!okw || rename(tmp.c_str(), path) != 0) {
        (void)remove(tmp.c_str());
        return fail(CCQ_E_INVALID, "cannot write %s: %s", path, strerror(errno));
    }
    if (n_entries) *n_entries = n;
    return ok();
}

}  // extern "C"
