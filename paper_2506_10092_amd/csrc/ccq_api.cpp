// Host side of the ccq C-ABI (include/ccq.h): validation, plan compilation
// (predicate folding, code tables, tiling, LDS layout) and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "ccq_internal.h"

using namespace ccq;

namespace ccq {
const char* last_error();
}

namespace ccq {

namespace {
thread_local std::string g_err;
}

ccq_status fail(ccq_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

ccq_status ok() {
    g_err.clear();
    return CCQ_OK;
}

ccq_status hip_fail(hipError_t e, const char* what) {
    return fail(CCQ_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

}  // namespace ccq

extern "C" {

const char* ccq_last_error(void) { return ccq::last_error(); }

int32_t ccq_abi_version(void) { return CCQ_ABI_VERSION; }

ccq_status ccq_context_create(int32_t device, ccq_context** out) {
    if (!out) return fail(CCQ_E_INVALID, "out is NULL");
    *out = nullptr;
    if (device == CCQ_HOST_ONLY) {
        ccq_context* c = new (std::nothrow) ccq_context;
        if (!c) return fail(CCQ_E_NOMEM, "out of host memory");
        c->device = -1;
        c->cus = 256;
        c->lds_per_block = 160 * 1024;
        c->scratch = nullptr;
        c->arch = "host";
        *out = c;
        return ok();
    }
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(CCQ_E_INVALID, "device %d out of range (%d devices)", device, n);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
        return fail(CCQ_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
    // the fixed scratch's address on this device (each device holds its own copy)
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    void* scratch = nullptr;
    e = scratch_address(&scratch);
    if (e != hipSuccess || !scratch) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    ccq_context* c = new (std::nothrow) ccq_context;
    if (!c) return fail(CCQ_E_NOMEM, "out of host memory");
    c->device = device;
    c->cus = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    c->scratch = scratch;
    c->arch = prop.gcnArchName;
    *out = c;
    return ok();
}

void ccq_context_destroy(ccq_context* ctx) { delete ctx; }

ccq_status ccq_table_create(ccq_context* ctx, int64_t n_rows, const ccq_column_desc* cols, int32_t n_cols,
                            ccq_table** out) {
    if (!out) return fail(CCQ_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(CCQ_E_INVALID, "context is NULL");
    if (n_rows < 0) return fail(CCQ_E_INVALID, "n_rows must be >= 0");
    if (n_cols < 0 || (n_cols > 0 && !cols)) return fail(CCQ_E_INVALID, "bad column array");
    for (int i = 0; i < n_cols; ++i) {
        const ccq_column_desc& c = cols[i];
        const bool comp = c.encoding == CCQ_RLE_INDEX || c.encoding == CCQ_PLAIN_INDEX;
        if (comp) {
            // the Index part of a composite column
            if (c.position_type != CCQ_I32 && c.position_type != CCQ_I64)
                return fail(CCQ_E_INVALID, "column %d: point position_type must be CCQ_I32 or CCQ_I64", i);
            if (c.value_type != CCQ_I32 && c.value_type != CCQ_I64)
                return fail(CCQ_E_INVALID, "column %d: value_type must be CCQ_I32 or CCQ_I64", i);
            if (c.n_points < 0 || c.n_points > n_rows)
                return fail(CCQ_E_INVALID, "column %d: n_points out of range", i);
            if (c.position_type == CCQ_I32 && n_rows > (int64_t)INT32_MAX + 1)
                return fail(CCQ_E_INVALID, "column %d: int32 positions cannot address %lld rows", i,
                            (long long)n_rows);
            if (c.n_points > 0 && (!c.point_values || !c.positions))
                return fail(CCQ_E_INVALID, "column %d: point values / positions missing", i);
        } else if (c.n_points != 0) {
            return fail(CCQ_E_INVALID, "column %d: n_points is for composite columns only", i);
        }
        if (c.encoding == CCQ_RLE || c.encoding == CCQ_RLE_INDEX) {
            if (c.value_type != CCQ_I32 && c.value_type != CCQ_I64)
                return fail(CCQ_E_INVALID, "column %d: RLE value_type must be CCQ_I32 or CCQ_I64", i);
            if (n_rows > 0 && c.n_entries < 1) return fail(CCQ_E_INVALID, "column %d: RLE column needs runs", i);
            if (c.n_entries > n_rows) return fail(CCQ_E_INVALID, "column %d: more runs than rows", i);
            if (c.n_entries > 0 && (!c.values || !c.run_ends))
                return fail(CCQ_E_INVALID, "column %d: RLE values / run_ends missing", i);
        } else if (c.encoding == CCQ_INDEX) {
            if (c.value_type != CCQ_I32 && c.value_type != CCQ_I64)
                return fail(CCQ_E_INVALID, "column %d: INDEX value_type must be CCQ_I32 or CCQ_I64", i);
            if (c.position_type != CCQ_I32 && c.position_type != CCQ_I64)
                return fail(CCQ_E_INVALID, "column %d: INDEX position_type must be CCQ_I32 or CCQ_I64", i);
            if (c.n_entries < 0 || c.n_entries > n_rows)
                return fail(CCQ_E_INVALID, "column %d: INDEX n_entries out of range", i);
            if (c.position_type == CCQ_I32 && n_rows > (int64_t)INT32_MAX + 1)
                return fail(CCQ_E_INVALID, "column %d: int32 positions cannot address %lld rows", i,
                            (long long)n_rows);
            if (c.n_entries > 0 && (!c.values || !c.positions))
                return fail(CCQ_E_INVALID, "column %d: INDEX values / positions missing", i);
        } else if (c.encoding == CCQ_BITPACKED || c.encoding == CCQ_PLAIN_INDEX) {
            if (c.bit_width < 1 || c.bit_width > 32)
                return fail(CCQ_E_INVALID, "column %d: bit_width must be in 1..32", i);
            if (c.n_entries != n_rows) return fail(CCQ_E_INVALID, "column %d: BITPACKED n_entries must equal n_rows", i);
            if (n_rows > 0 && !c.packed) return fail(CCQ_E_INVALID, "column %d: packed stream missing", i);
        } else {
            return fail(CCQ_E_INVALID, "column %d: unknown encoding %d", i, c.encoding);
        }
        if (c.dict_values ? (c.encoding != CCQ_BITPACKED || c.dict_size < 1) : c.dict_size != 0)
            return fail(CCQ_E_INVALID,
                        "column %d: a dictionary needs a BITPACKED column and dict_size >= 1 (dict_size 0 without one)",
                        i);
    }
    ccq_table* t = new (std::nothrow) ccq_table;
    if (!t) return fail(CCQ_E_NOMEM, "out of host memory");
    t->ctx = ctx;
    t->n_rows = n_rows;
    t->cols.assign(cols, cols + n_cols);
    *out = t;
    return ok();
}

void ccq_table_destroy(ccq_table* t) { delete t; }

ccq_status ccq_table_validate(ccq_table* t, void* stream) {
    if (!t) return fail(CCQ_E_INVALID, "table is NULL");
    if (t->ctx->device < 0) return fail(CCQ_E_UNSUPPORTED, "host-only context has no device");
    hipError_t e = hipSetDevice(t->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const size_t nc = std::max<size_t>(t->cols.size(), 1);
    int32_t* flag = nullptr;                    // one flag per column
    e = hipMalloc(&flag, sizeof(int32_t) * nc);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    std::vector<int32_t> host(nc, 0);
    e = hipMemcpyAsync(flag, host.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, s);
    for (size_t i = 0; i < t->cols.size() && e == hipSuccess; ++i) {
        const ccq_column_desc& c = t->cols[i];
        if ((c.encoding == CCQ_RLE || c.encoding == CCQ_RLE_INDEX) && c.n_entries > 0)
            e = launch_validate_rle(c.run_ends, c.n_entries, t->n_rows, flag + i, s);
        if (c.encoding == CCQ_INDEX && c.n_entries > 0)
            e = launch_validate_idx(c.positions, c.position_type, c.n_entries, t->n_rows, flag + i, s);
        if (e == hipSuccess && c.n_points > 0)
            e = launch_validate_idx(c.positions, c.position_type, c.n_points, t->n_rows, flag + i, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), flag, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(flag);
    if (e != hipSuccess) return hip_fail(e, "table validation");
    for (size_t i = 0; i < t->cols.size(); ++i)
        if (host[i]) return fail(CCQ_E_INVALID, "column %zu: run ends or positions are not valid", i);
    return ok();
}

}  // extern "C"

// ------------------------------------------------------------------ plan compilation

namespace {

// Values as sorted, disjoint inclusive intervals: the conjunction of plain
// and negated RANGE / IN predicates on one column is one such list.
typedef std::vector<std::pair<int64_t, int64_t>> Intervals;

Intervals iv_of_range(int64_t lo, int64_t hi) {   // lo <= v < hi
    if (lo >= hi) return {};
    return {{lo, hi - 1}};
}

Intervals iv_of_set(const std::set<int64_t>& s) {
    Intervals r;
    for (int64_t v : s) {
        if (!r.empty() && r.back().second != INT64_MAX && r.back().second + 1 == v) r.back().second = v;
        else r.push_back({v, v});
    }
    return r;
}

Intervals iv_complement(const Intervals& a) {
    Intervals r;
    int64_t next = INT64_MIN;    // lowest value not yet covered
    bool open = true;            // values from `next` on are still to place
    for (const auto& x : a) {
        if (x.first > next) r.push_back({next, x.first - 1});
        if (x.second == INT64_MAX) {
            open = false;
            break;
        }
        next = x.second + 1;
    }
    if (open) r.push_back({next, INT64_MAX});
    return r;
}

Intervals iv_intersect(const Intervals& a, const Intervals& b) {
    Intervals r;
    size_t i = 0, j = 0;
    while (i < a.size() && j < b.size()) {
        const int64_t lo = std::max(a[i].first, b[j].first), hi = std::min(a[i].second, b[j].second);
        if (lo <= hi) r.push_back({lo, hi});
        if (a[i].second < b[j].second) ++i; else ++j;
    }
    return r;
}

Intervals iv_union(const Intervals& a, const Intervals& b) {
    return iv_complement(iv_intersect(iv_complement(a), iv_complement(b)));
}

bool iv_all(const Intervals& a) {
    return a.size() == 1 && a[0].first == INT64_MIN && a[0].second == INT64_MAX;
}

// the values a predicate passes
ccq_status pred_intervals(const ccq_pred& p, int i, Intervals& a) {
    if (p.op == CCQ_RANGE || p.op == CCQ_NOT_RANGE) {
        a = iv_of_range(p.lo, p.hi);
    } else if (p.op == CCQ_IN || p.op == CCQ_NOT_IN) {
        if (p.in_len < 0 || (p.in_len > 0 && !p.in_list)) return fail(CCQ_E_INVALID, "predicate %d: bad IN list", i);
        a = iv_of_set(std::set<int64_t>(p.in_list, p.in_list + p.in_len));
    } else {
        return fail(CCQ_E_INVALID, "predicate %d: unknown op %d", i, p.op);
    }
    if (p.op == CCQ_NOT_RANGE || p.op == CCQ_NOT_IN) a = iv_complement(a);   // NOT (Section 5.3)
    return CCQ_OK;
}

struct Fold {               // conjunction of predicates on one column
    bool constrained = false;
    Intervals iv;             // the passing values, when constrained
    // the same, in the simplest form the kernels take
    bool has_range = false, has_set = false, has_iv = false, is_false = false;
    bool has_not_range = false;   // every value outside [lo, hi)
    int64_t lo = 0, hi = 0;   // [lo, hi) when has_range
    std::set<int64_t> set;
};

// the simplest form of a column's passing values: nothing, one half-open
// range, a set of single values, or a list of intervals
void fold_classify(Fold& f) {
    if (f.constrained && iv_all(f.iv)) f.constrained = false;
    if (!f.constrained) return;
    if (f.iv.empty()) {
        f.is_false = true;
    } else if (f.iv.size() == 1 && f.iv[0].second != INT64_MAX) {
        f.has_range = true;
        f.lo = f.iv[0].first;
        f.hi = f.iv[0].second + 1;
    } else if (f.iv.size() == 1) {               // [lo, INT64_MAX]: outside [INT64_MIN, lo)
        f.has_not_range = true;
        f.lo = INT64_MIN;
        f.hi = f.iv[0].first;
    } else if (f.iv.size() == 2 && f.iv[0].first == INT64_MIN && f.iv[1].second == INT64_MAX) {
        f.has_not_range = true;                  // the complement of one range (NOT, Section 5.3)
        f.lo = f.iv[0].second + 1;
        f.hi = f.iv[1].first;
    } else {
        bool single = true;
        for (const auto& x : f.iv) single = single && x.first == x.second;
        if (single) {
            f.has_set = true;
            for (const auto& x : f.iv) f.set.insert(x.first);
        } else {
            f.has_iv = true;
        }
    }
}

bool fold_pass(const Fold& f, int64_t v) {
    if (!f.constrained) return true;
    // first interval whose low end is > v
    auto it = std::upper_bound(f.iv.begin(), f.iv.end(), std::make_pair(v, INT64_MAX));
    return it != f.iv.begin() && v <= std::prev(it)->second;
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

struct Compiled {
    DevPlan P;
    std::vector<unsigned char> blob;        // DevPlan followed by tables, sets, slot keys
    std::vector<std::pair<size_t, size_t>> fixes;   // (pointer field offset in DevPlan, data offset in blob)
};

ccq_status compile_plan(const ccq_table* t, const ccq_query_desc* q, Compiled& out) {
    if (!t || !q) return fail(CCQ_E_INVALID, "table or query is NULL");
    const int ncol = (int)t->cols.size();
    if (q->n_preds < 0 || q->n_keys < 0 || q->n_aggs < 0) return fail(CCQ_E_INVALID, "negative counts");
    if ((q->n_preds && !q->preds) || (q->n_keys && !q->keys) || (q->n_aggs && !q->aggs))
        return fail(CCQ_E_INVALID, "query arrays missing");
    if (q->row_begin < 0 || q->row_end > t->n_rows || q->row_begin > q->row_end)
        return fail(CCQ_E_INVALID, "window [%lld, %lld) outside the table of %lld rows", (long long)q->row_begin,
                    (long long)q->row_end, (long long)t->n_rows);
    if (q->n_keys > kMaxKeys) return fail(CCQ_E_UNSUPPORTED, "at most %d group keys", kMaxKeys);
    if (q->n_aggs > kMaxAggs) return fail(CCQ_E_UNSUPPORTED, "at most %d aggregates", kMaxAggs);

    DevPlan& P = out.P;
    memset(&P, 0, sizeof P);
    P.off_rcl = -1;       // no row clause unless the layout below places one
    P.row_begin = q->row_begin;
    P.row_end = q->row_end;

    // referenced columns, grouped by encoding, in order of first use
    // a composite column (Section 3.2) takes the slot of its base part (RLE
    // or bit-packed) plus a CompCol for its points
    auto base_enc = [&](int c) {
        const int enc = t->cols[c].encoding;
        return enc == CCQ_RLE_INDEX ? CCQ_RLE : enc == CCQ_PLAIN_INDEX ? CCQ_BITPACKED : enc;
    };
    auto is_comp = [&](int c) {
        return t->cols[c].encoding == CCQ_RLE_INDEX || t->cols[c].encoding == CCQ_PLAIN_INDEX;
    };
    std::vector<int> kind_slot(ncol, -1);
    std::vector<int> rle_cols, bp_cols, idx_cols, comp_cols;
    auto use = [&](int c) -> ccq_status {
        if (c < 0 || c >= ncol) return fail(CCQ_E_INVALID, "column index %d out of range", c);
        if (kind_slot[c] >= 0) return CCQ_OK;
        int enc = base_enc(c);
        std::vector<int>& v = enc == CCQ_RLE ? rle_cols : enc == CCQ_BITPACKED ? bp_cols : idx_cols;
        kind_slot[c] = (int)v.size();
        v.push_back(c);
        if (is_comp(c)) comp_cols.push_back(c);
        return CCQ_OK;
    };
    for (int i = 0; i < q->n_preds; ++i) {
        const ccq_pred& p = q->preds[i];
        if (p.col < 0 || p.col >= ncol) return fail(CCQ_E_INVALID, "predicate %d: column %d out of range", i, p.col);
        if (p.clause < 0) return fail(CCQ_E_INVALID, "predicate %d: clause must be >= 0", i);
    }
    // clause-0 predicates, keys and SUMs use the columns' own slots
    for (int i = 0; i < q->n_preds; ++i)
        if (q->preds[i].clause == 0)
            if (ccq_status s = use(q->preds[i].col)) return s;
    for (int i = 0; i < q->n_keys; ++i)
        if (ccq_status s = use(q->keys[i].col)) return s;
    for (int i = 0; i < q->n_aggs; ++i) {
        const ccq_agg& ag = q->aggs[i];
        if (ag.func == CCQ_SUM || ag.func == CCQ_MIN || ag.func == CCQ_MAX) {
            if (ag.op < CCQ_OP_NONE || ag.op > CCQ_OP_MUL)
                return fail(CCQ_E_INVALID, "aggregate %d: unknown operator %d", i, ag.op);
            if (ccq_status s = use(ag.col)) return s;
            if (ag.op != CCQ_OP_NONE)
                if (ccq_status s = use(ag.col2)) return s;
        } else if (ag.func != CCQ_COUNT_STAR) {
            return fail(CCQ_E_INVALID, "aggregate %d: unknown function %d", i, ag.func);
        }
    }

    // fold the clause-0 predicates per column (AND: composite predicates on
    // one column become one list of intervals)
    std::vector<Fold> fold(ncol);
    for (int i = 0; i < q->n_preds; ++i) {
        const ccq_pred& p = q->preds[i];
        if (p.clause != 0) continue;
        Intervals a;
        if (ccq_status s = pred_intervals(p, i, a)) return s;
        Fold& f = fold[p.col];
        f.iv = f.constrained ? iv_intersect(f.iv, a) : a;
        f.constrained = true;
    }
    // OR clauses (Section 5.2): per clause and column, the union of the
    // predicates' intervals.  A clause over one column is one more AND on
    // that column; a clause over several RLE columns gets a slot per column,
    // consecutive, whose pass masks the kernels OR
    struct Clause {
        int32_t id;
        std::vector<int> cols;
        std::vector<Intervals> iv;
    };
    std::vector<Clause> clauses;
    for (int i = 0; i < q->n_preds; ++i) {
        const ccq_pred& p = q->preds[i];
        if (p.clause == 0) continue;
        Intervals a;
        if (ccq_status s = pred_intervals(p, i, a)) return s;
        size_t k = 0;
        while (k < clauses.size() && clauses[k].id != p.clause) ++k;
        if (k == clauses.size()) clauses.push_back({p.clause, {}, {}});
        Clause& cl = clauses[k];
        size_t j = 0;
        while (j < cl.cols.size() && cl.cols[j] != p.col) ++j;
        if (j == cl.cols.size()) {
            cl.cols.push_back(p.col);
            cl.iv.push_back(a);
        } else {
            cl.iv[j] = iv_union(cl.iv[j], a);
        }
    }
    struct OrSlot {
        int col;
        Fold f;
        bool or_next;
        bool row_clause;
    };
    std::vector<OrSlot> or_slots;
    // at most one clause over RLE and bit-packed columns (RLE mask OR Plain
    // mask, Table 4): its RLE part is a mask of its own, and each row of it
    // is tested against the bit-packed part
    bool row_clause = false;
    std::vector<std::pair<int, Intervals>> bp_or;
    // an OR clause over RLE columns and one Index column: the Index part's
    // column and intervals (the clause is the row clause, applied to the row
    // mask once the Index points are known)
    int idx_or_col = -1;
    Intervals idx_or_iv;
    int false_col = -1;    // a clause no row can pass: the query is false
    for (const Clause& cl : clauses) {
        std::vector<size_t> live;
        bool always = false;
        for (size_t j = 0; j < cl.cols.size(); ++j) {
            if (iv_all(cl.iv[j])) always = true;
            else if (!cl.iv[j].empty()) live.push_back(j);
        }
        if (always) continue;
        if (live.empty()) {
            if (false_col < 0) false_col = cl.cols[0];
            continue;
        }
        if (live.size() == 1) {
            const int c = cl.cols[live[0]];
            Fold& f = fold[c];
            f.iv = f.constrained ? iv_intersect(f.iv, cl.iv[live[0]]) : cl.iv[live[0]];
            f.constrained = true;
            if (ccq_status s = use(c)) return s;
            continue;
        }
        bool mixed = false;
        int n_index = 0, index_j = -1;
        for (size_t j : live) {
            if (is_comp(cl.cols[j]))
                return fail(CCQ_E_UNSUPPORTED, "OR clause %d: an OR across columns takes no composite column", cl.id);
            if (t->cols[cl.cols[j]].encoding == CCQ_INDEX) {
                ++n_index;
                index_j = (int)j;
            }
            mixed = mixed || t->cols[cl.cols[j]].encoding == CCQ_BITPACKED;
        }
        if (n_index > 0) {
            // RLE columns OR one Index column (Table 4, RLE mask OR Index mask)
            if (n_index > 1 || mixed)
                return fail(CCQ_E_UNSUPPORTED,
                            "OR clause %d: an OR across columns takes at most one INDEX column, with RLE columns only",
                            cl.id);
            if (row_clause)
                return fail(CCQ_E_UNSUPPORTED, "OR clause %d: at most one OR clause may name INDEX or bit-packed "
                                               "columns beside RLE ones", cl.id);
            row_clause = true;
            idx_or_col = cl.cols[index_j];
            idx_or_iv = cl.iv[index_j];
        }
        if (mixed) {
            if (row_clause)
                return fail(CCQ_E_UNSUPPORTED, "OR clause %d: at most one OR clause may span RLE and bit-packed columns",
                            cl.id);
            row_clause = true;
        }
        std::vector<size_t> rle_live;
        for (size_t j : live) {
            if (t->cols[cl.cols[j]].encoding == CCQ_INDEX) continue;
            if (t->cols[cl.cols[j]].encoding == CCQ_RLE) {
                rle_live.push_back(j);
            } else {
                bp_or.push_back({cl.cols[j], cl.iv[j]});
                if (ccq_status s = use(cl.cols[j])) return s;
            }
        }
        for (size_t n = 0; n < rle_live.size(); ++n) {
            OrSlot o;
            o.col = cl.cols[rle_live[n]];
            o.f.constrained = true;
            o.f.iv = cl.iv[rle_live[n]];
            fold_classify(o.f);
            o.or_next = n + 1 < rle_live.size();
            o.row_clause = mixed || n_index > 0;
            or_slots.push_back(o);
        }
    }
    if (false_col >= 0) {
        if (ccq_status s = use(false_col)) return s;
        fold[false_col].constrained = true;
        fold[false_col].iv.clear();
    }
    if ((int)(rle_cols.size() + or_slots.size()) > kMaxRle)
        return fail(CCQ_E_UNSUPPORTED, "at most %d RLE column uses per query (one per column, plus one per OR clause naming it)", kMaxRle);
    if ((int)bp_cols.size() > kMaxBp)
        return fail(CCQ_E_UNSUPPORTED, "at most %d bit-packed columns per query", kMaxBp);
    if ((int)idx_cols.size() + (idx_or_col >= 0 ? 1 : 0) > kMaxIdx)
        return fail(CCQ_E_UNSUPPORTED, "at most %d Index columns per query (an OR clause's Index column counts once "
                                       "more)", kMaxIdx);
    if ((int)comp_cols.size() > kMaxComp)
        return fail(CCQ_E_UNSUPPORTED, "at most %d composite columns per query", kMaxComp);
    for (auto& f : fold) fold_classify(f);
    // a composite column's predicates are tested per row on its value (the
    // point's or the base part's), so its base part gets none
    Fold no_pred;
    fold_classify(no_pred);
    auto base_fold = [&](int c) -> const Fold& { return is_comp(c) ? no_pred : fold[c]; };

    // device blob contents, laid out after the DevPlan
    std::vector<unsigned char>& blob = out.blob;
    blob.assign(align16(sizeof(DevPlan)), 0);
    auto blob_put = [&](const void* data, size_t bytes) -> size_t {
        size_t off = blob.size();
        blob.resize(align16(off + bytes));
        if (bytes) memcpy(blob.data() + off, data, bytes);
        return off;
    };
    auto fix_ptr = [&](const void* field, size_t data_off) {
        out.fixes.push_back({(size_t)((const unsigned char*)field - (const unsigned char*)&P), data_off});
    };

    P.k_rle = (int)(rle_cols.size() + or_slots.size());
    P.n_bp = (int)bp_cols.size();
    P.n_idx = (int)idx_cols.size() + (idx_or_col >= 0 ? 1 : 0);
    // a column's folded predicate in the form the kernels test
    auto put_pred = [&](const Fold& f, int32_t& pred, int64_t& lo, int64_t& hi, const int64_t*& set,
                        int32_t& set_len) {
        if (f.is_false) pred = kPredFalse;
        else if (f.has_set) {
            pred = kPredSet;
            std::vector<int64_t> v(f.set.begin(), f.set.end());
            set_len = (int32_t)v.size();
            fix_ptr(&set, blob_put(v.data(), v.size() * 8));
        } else if (f.has_iv) {
            pred = kPredIntervals;
            std::vector<int64_t> v;
            for (const auto& x : f.iv) {
                v.push_back(x.first);
                v.push_back(x.second);
            }
            set_len = (int32_t)f.iv.size();
            fix_ptr(&set, blob_put(v.data(), v.size() * 8));
        } else if (f.has_range) {
            pred = kPredRange;
            lo = f.lo;
            hi = f.hi;
        } else if (f.has_not_range) {
            pred = kPredNotRange;
            lo = f.lo;
            hi = f.hi;
        } else pred = kPredNone;
    };
    for (int s = 0; s < P.k_rle; ++s) {
        const bool own = s < (int)rle_cols.size();
        const OrSlot* o = own ? nullptr : &or_slots[s - rle_cols.size()];
        const ccq_column_desc& c = t->cols[own ? rle_cols[s] : o->col];
        const Fold& f = own ? base_fold(rle_cols[s]) : o->f;
        RleCol& r = P.rle[s];
        r.or_next = (o && o->or_next) ? 1 : 0;
        r.row_clause = (o && o->row_clause) ? 1 : 0;
        r.sum_slot = -1;
        r.ends = c.run_ends;
        r.vals = c.values;
        r.n_runs = c.n_entries;
        r.vtype = c.value_type;
        put_pred(f, r.pred, r.lo, r.hi, r.set, r.set_len);
    }
    bool idx_pred = false;
    for (int s = 0; s < (int)idx_cols.size(); ++s) {
        const ccq_column_desc& c = t->cols[idx_cols[s]];
        IdxCol& x = P.idx[s];
        x.pos = c.positions;
        x.vals = c.values;
        x.n = c.n_entries;
        x.ptype = c.position_type;
        x.vtype = c.value_type;
        x.sum_slot = -1;
        // an Index column's value is 0 at the rows it does not list
        const Fold& f = fold[idx_cols[s]];
        put_pred(f, x.pred, x.lo, x.hi, x.set, x.set_len);
        x.zero_pass = fold_pass(f, 0) ? 1 : 0;
        idx_pred = idx_pred || x.pred != kPredNone;
    }
    if (idx_or_col >= 0) {
        // the OR clause's Index part: a slot of its own, its mask ORed with the
        // clause's RLE part (the row clause word) before the row mask takes it
        const ccq_column_desc& c = t->cols[idx_or_col];
        IdxCol& x = P.idx[P.n_idx - 1];
        x.pos = c.positions;
        x.vals = c.values;
        x.n = c.n_entries;
        x.ptype = c.position_type;
        x.vtype = c.value_type;
        x.sum_slot = -1;
        Fold f;
        f.constrained = true;
        f.iv = idx_or_iv;
        fold_classify(f);
        put_pred(f, x.pred, x.lo, x.hi, x.set, x.set_len);
        x.zero_pass = fold_pass(f, 0) ? 1 : 0;
        x.or_rcl = 1;
        idx_pred = true;
    }

    // keys: mixed radix; bit-packed keys up to kLutMaxBits bits get dense
    // slots over the key values their passing codes can reach
    P.n_keys = q->n_keys;
    std::vector<std::vector<int64_t>> slot_keys(q->n_keys);
    std::vector<int> bp_key(P.n_bp, -1);
    for (int k = 0; k < q->n_keys; ++k) {
        const ccq_key& key = q->keys[k];
        const ccq_column_desc& c = t->cols[key.col];
        if (is_comp(key.col))
            return fail(CCQ_E_UNSUPPORTED, "key %d: group keys on composite columns are not supported", k);
        if (key.shift < 0 || key.shift > 62) return fail(CCQ_E_INVALID, "key %d: shift must be in 0..62", k);
        if (key.card < 1) return fail(CCQ_E_INVALID, "key %d: card must be >= 1", k);
        KeyDesc& kd = P.keys[k];
        kd.shift = key.shift;
        kd.card = key.card;
        kd.src = kind_slot[key.col];
        if (c.encoding == CCQ_RLE) {
            kd.src_kind = kKeyRle;
            kd.radix = key.card;
            RleCol& r = P.rle[kd.src];
            if (r.key_on) return fail(CCQ_E_UNSUPPORTED, "key %d: an RLE column may be one group key only", k);
            r.key_on = 1;
            r.key_shift = key.shift;
            r.key_card = key.card;
        } else if (c.encoding == CCQ_BITPACKED) {
            kd.src_kind = kKeyBp;
            if (c.dict_values) {
                if (key.shift != 0 || key.card > c.dict_size)
                    return fail(CCQ_E_INVALID,
                                "key %d: a key on a dictionary column needs shift 0 and card <= dict_size (%lld)", k,
                                (long long)c.dict_size);
                kd.dict = c.dict_values;
            }
            if (bp_key[kd.src] >= 0)
                return fail(CCQ_E_UNSUPPORTED, "key %d: a bit-packed column may be one group key only", k);
            bp_key[kd.src] = k;
            if (c.bit_width <= kLutMaxBits) {
                kd.via_lut = 1;
                const Fold& f = fold[key.col];
                std::set<int64_t> reach;
                for (int64_t code = 0; code < (int64_t(1) << c.bit_width); ++code) {
                    int64_t v = c.base + code;
                    if (!fold_pass(f, v)) continue;
                    int64_t kv = v >> key.shift;
                    if (kv >= 0 && kv < key.card) reach.insert(kv);
                }
                slot_keys[k].assign(reach.begin(), reach.end());
                kd.radix = std::max<int64_t>(1, (int64_t)slot_keys[k].size());
                if (slot_keys[k].empty()) slot_keys[k].push_back(0);
                fix_ptr(&kd.slot_keys, blob_put(slot_keys[k].data(), slot_keys[k].size() * 8));
            } else {
                kd.radix = key.card;
            }
        } else {
            return fail(CCQ_E_UNSUPPORTED, "key %d: group keys on INDEX columns are not supported", k);
        }
    }
    int64_t G = 1;
    for (int k = q->n_keys - 1; k >= 0; --k) {
        P.keys[k].stride = G;
        if (P.keys[k].radix > kMaxGroups / G)
            return fail(CCQ_E_UNSUPPORTED, "more than 2^27 key combinations (product of key domains)");
        G *= P.keys[k].radix;
    }
    P.n_groups = G;
    for (int k = 0; k < q->n_keys; ++k)
        if (P.keys[k].src_kind == kKeyRle) P.rle[P.keys[k].src].key_stride = P.keys[k].stride;

    // bit-packed columns: predicates and key slots folded into one code table
    // per column (built here, encoded once the kernel path is known)
    std::vector<std::vector<uint16_t>> lut16(P.n_bp);
    for (int s = 0; s < P.n_bp; ++s) {
        const ccq_column_desc& c = t->cols[bp_cols[s]];
        const Fold& f = base_fold(bp_cols[s]);
        BpCol& b = P.bp[s];
        b.packed = c.packed;
        b.base = c.base;
        b.w = c.bit_width;
        b.key = bp_key[s];
        b.sum_slot = -1;
        if (b.key >= 0) {
            b.key_shift = P.keys[b.key].shift;
            b.key_card = P.keys[b.key].card;
            b.key_stride = P.keys[b.key].stride;
        }
        const bool has_pred = f.constrained;
        b.n_words = (t->n_rows * (int64_t)c.bit_width + 31) / 32 + 2;
        if (c.bit_width <= kLutMaxBits && (has_pred || b.key >= 0)) {
            const int64_t n = int64_t(1) << c.bit_width;
            std::vector<uint16_t>& lut = lut16[s];
            lut.assign(n, kLutReject);
            std::map<int64_t, int64_t> rank;
            if (b.key >= 0)
                for (size_t i = 0; i < slot_keys[b.key].size(); ++i) rank[slot_keys[b.key][i]] = (int64_t)i;
            for (int64_t code = 0; code < n; ++code) {
                const int64_t v = c.base + code;
                if (!fold_pass(f, v)) continue;
                if (b.key < 0) { lut[code] = 0; continue; }
                const KeyDesc& kd = P.keys[b.key];
                const int64_t kv = v >> kd.shift;
                lut[code] = (kv < 0 || kv >= kd.card) ? kLutDomain : (uint16_t)rank[kv];
            }
        } else {
            put_pred(f, b.pred, b.lo, b.hi, b.set, b.set_len);
        }
    }

    // the bit-packed part of the row clause, per column
    for (int s = 0; s < P.n_bp; ++s) {
        BpCol& b = P.bp[s];
        b.or_pred = kPredNone;
        for (const auto& m : bp_or) {
            if (m.first != bp_cols[s]) continue;
            Fold f;
            f.constrained = true;
            f.iv = m.second;
            fold_classify(f);
            put_pred(f, b.or_pred, b.or_lo, b.or_hi, b.or_set, b.or_set_len);
            if (b.w <= kLutMaxBits) {
                // one bit per code: the code's value passes this column's part of the clause
                std::vector<uint32_t> bits(((size_t(1) << b.w) + 31) / 32, 0u);
                for (int64_t code = 0; code < (int64_t(1) << b.w); ++code)
                    if (fold_pass(f, b.base + code)) bits[code >> 5] |= 1u << (code & 31);
                b.or_bits_words = (int32_t)bits.size();
                fix_ptr(&b.or_bits, blob_put(bits.data(), bits.size() * 4));
            }
        }
    }

    // aggregates.  A plan with MIN, MAX or a two-column expression gives
    // every aggregate but COUNT and an Index column's SUM an ExtAcc
    // (accumulators [0, n_ext)), evaluated per row on the generic row path.
    P.n_aggs = q->n_aggs;
    bool ext = false;
    for (int a = 0; a < q->n_aggs; ++a)
        ext = ext || q->aggs[a].func == CCQ_MIN || q->aggs[a].func == CCQ_MAX || q->aggs[a].op != CCQ_OP_NONE;
    std::vector<char> placed(q->n_aggs, 0);
    for (int a = 0; ext && a < q->n_aggs; ++a) {
        const ccq_agg& ag = q->aggs[a];
        AggDesc& ad = P.aggs[a];
        ad.fin = kFinValue;
        if (ag.func == CCQ_COUNT_STAR) {
            ad.kind = kAggCount;
            ad.sum_slot = -1;
            placed[a] = 1;
            continue;
        }
        if (ag.func == CCQ_SUM && ag.op == CCQ_OP_NONE && t->cols[ag.col].encoding == CCQ_INDEX) continue;
        const int opnd[2] = {ag.col, ag.op != CCQ_OP_NONE ? ag.col2 : ag.col};
        for (int k = 0; k < 2; ++k) {
            const ccq_column_desc& c = t->cols[opnd[k]];
            if (c.encoding == CCQ_INDEX)
                return fail(CCQ_E_UNSUPPORTED, "aggregate %d: MIN, MAX and expressions take RLE and BITPACKED columns",
                            a);
            if (c.dict_values)
                return fail(CCQ_E_UNSUPPORTED, "aggregate %d: over a dictionary-encoded column", a);
        }
        const int slot = P.n_sums++;
        ExtAcc& e = P.ext[slot];
        e.kind = ag.func == CCQ_MIN ? kExtMin : ag.func == CCQ_MAX ? kExtMax : kExtSum;
        e.op = ag.op;
        e.a_rle = base_enc(opnd[0]) == CCQ_RLE ? 1 : 0;
        e.a_src = kind_slot[opnd[0]];
        e.b_rle = base_enc(opnd[1]) == CCQ_RLE ? 1 : 0;
        e.b_src = kind_slot[opnd[1]];
        if (e.a_rle) P.rle[e.a_src].keep_value = 1;
        if (e.b_rle) P.rle[e.b_src].keep_value = 1;
        ad.kind = kAggExt;
        ad.src = slot;
        ad.sum_slot = slot;
        ad.fin = e.kind == kExtMin ? kFinMin : e.kind == kExtMax ? kFinMax : kFinValue;
        placed[a] = 1;
    }
    P.n_ext = P.n_sums;
    for (int a = 0; a < q->n_aggs; ++a) {
        AggDesc& ad = P.aggs[a];
        if (placed[a]) continue;
        ad.fin = kFinValue;
        if (q->aggs[a].func == CCQ_COUNT_STAR) {
            ad.kind = kAggCount;
            ad.sum_slot = -1;
            continue;
        }
        const int col = q->aggs[a].col;
        const int enc = base_enc(col);
        if (t->cols[col].dict_values)
            return fail(CCQ_E_UNSUPPORTED, "aggregate %d: SUM over a dictionary-encoded column", a);
        ad.kind = enc == CCQ_RLE ? kAggSumRle : enc == CCQ_BITPACKED ? kAggSumBp : kAggSumIdx;
        ad.src = kind_slot[col];
        // one accumulator per column: repeated SUMs of a column share it
        int32_t& slot = enc == CCQ_RLE ? P.rle[ad.src].sum_slot
                        : enc == CCQ_BITPACKED ? P.bp[ad.src].sum_slot : P.idx[ad.src].sum_slot;
        if (slot < 0) slot = P.n_sums++;
        ad.sum_slot = slot;
    }

    // composite columns: the points, and the predicate tested per row
    P.n_comp = (int32_t)comp_cols.size();
    for (int i = 0; i < P.n_comp; ++i) {
        const int col = comp_cols[i];
        const ccq_column_desc& c = t->cols[col];
        CompCol& cc = P.comp[i];
        cc.rle = base_enc(col) == CCQ_RLE ? 1 : 0;
        cc.src = kind_slot[col];
        cc.pos = c.positions;
        cc.vals = c.point_values;
        cc.n = c.n_points;
        cc.ptype = c.position_type;
        cc.vtype = c.value_type;
        put_pred(fold[col], cc.pred, cc.lo, cc.hi, cc.set, cc.set_len);
        if (cc.rle) P.rle[cc.src].keep_value = 1;     // the run's value, read per row
    }

    // mode and tiling
    P.row_mode = (P.n_bp > 0 || P.n_ext > 0 || P.n_comp > 0) ? 1 : 0;
    P.any_rle_row = 0;
    for (int k = 0; k < P.n_ext; ++k)
        if (P.ext[k].a_rle || P.ext[k].b_rle) P.any_rle_row = 1;
    for (int i = 0; i < P.n_comp; ++i)
        if (P.comp[i].rle) P.any_rle_row = 1;
    if (P.row_mode) {
        for (int k = 0; k < P.n_keys; ++k)
            if (P.keys[k].src_kind == kKeyRle) P.any_rle_row = 1;
        for (int a = 0; a < P.n_aggs; ++a)
            if (P.aggs[a].kind == kAggSumRle) P.any_rle_row = 1;
    }
    const int64_t window = P.row_end - P.row_begin;
    // 2048-row tiles, lane l owning rows [32l, 32l + 32) of the tile; each
    // column keeps at least 64 staged runs (a tile that would overflow ends
    // early, on a multiple of 32 rows).  Run mode stages more, as its columns
    // are the only data read.
    P.span = kRowSpan;
    // staged runs per column: twice the runs a tile holds on average (at
    // least 64), so tiles rarely end early; run mode stages a little more
    // (never more than the column's runs, and at most kMaxStagedRuns per
    // wave in all: a column that needs more ends its tiles early)
    P.run_cap = 0;
    {
        int64_t want[kMaxRle] = {0};
        int64_t total = 0;
        for (int s = 0; s < P.k_rle; ++s) {
            const double per_tile =
                (double)kRowTile * (double)P.rle[s].n_runs / (double)std::max<int64_t>(t->n_rows, 1);
            int64_t cap = (int64_t)(2.0 * per_tile) + (P.row_mode ? 16 : 32);
            cap = std::min<int64_t>(cap, P.rle[s].n_runs + 1);
            want[s] = std::max<int64_t>(64, (cap + 15) & ~int64_t(15));
            total += want[s];
        }
        for (int s = 0; s < P.k_rle; ++s) {
            int64_t cap = want[s];
            if (total > kMaxStagedRuns)
                cap = std::max<int64_t>(64, (want[s] * kMaxStagedRuns / total) & ~int64_t(15));
            P.rle[s].stage_base = P.run_cap;
            P.rle[s].stage_cap = (int32_t)cap;
            P.run_cap += (int32_t)cap;
        }
    }
    P.tile_rows = (int64_t)64 * P.span;
    // nominal tiles: multiples of tile_rows in absolute row numbers that meet the window
    P.n_tiles = window > 0 ? (P.row_end - 1) / P.tile_rows - P.row_begin / P.tile_rows + 1 : 0;

    // kernel path.  The fast row path: a single bit-packed column of a width
    // with a kernel instance, at most one Index column and no predicate on it, no RLE value per row, the column itself the only
    // key (or no key), a code table or a plain range test, and uint32 counts
    // that cannot overflow within one workgroup.
    P.kmax = P.k_rle <= 2 ? 2 : P.k_rle <= 4 ? 4 : 8;
    P.w0 = 0;
    P.fast_big = 0;
    {
        bool fast = P.row_mode && P.n_bp == 1 && P.n_idx <= 1 && !P.any_rle_row && fast_row_width(P.bp[0].w) &&
                    !idx_pred && !row_clause && P.n_ext == 0 && P.n_comp == 0;
        BpCol& b = P.bp[0];
        const Fold& f = fold[bp_cols.empty() ? 0 : bp_cols[0]];
        if (fast && b.key < 0 && P.n_keys > 0) fast = false;
        // workgroups: at least min(tiles / 4, one per CU); rows per workgroup bounded by that
        const int64_t min_blocks = std::max<int64_t>(1, std::min<int64_t>((P.n_tiles + 3) / 4, t->ctx->cus));
        const int64_t rows_per_wg = ((P.n_tiles + 4 * min_blocks - 1) / (4 * min_blocks)) * 4 * P.tile_rows;
        if (fast && rows_per_wg >= (int64_t)1 << 31) fast = false;
        // the replicated static count table holds (G + 2) << 3 words; beyond
        // that, one uint32 table of G + 2 counts in dynamic LDS, slots
        // computed from the code (no set predicate, contiguous reachable
        // keys), no SUM of the column itself
        bool big = false;
        if (fast && (G + 2) * 8 > kFastCntWords) {
            big = (G + 2) * 4 <= kFastBigBytes && b.sum_slot < 0 && !f.has_set && !f.has_iv && !f.has_not_range;
            if (big && b.key >= 0 && P.keys[b.key].via_lut) {
                const std::vector<int64_t>& sk = slot_keys[b.key];
                big = sk.back() - sk.front() + 1 == (int64_t)sk.size();
            }
            if (!big) fast = false;
        }
        if (fast && (lut16[0].empty() || big)) {
            if (!big && (b.pred == kPredSet || b.pred == kPredIntervals || b.pred == kPredNotRange)) fast = false;
            const bool is_false = big ? f.is_false : b.pred == kPredFalse;
            const bool has_range = big ? f.has_range : b.pred == kPredRange;
            const int64_t rlo = big ? f.lo : b.lo, rhi = big ? f.hi : b.hi;
            const int64_t ncode = int64_t(1) << b.w;
            int64_t clo = 0, chi = ncode;
            if (is_false) chi = 0;
            if (has_range) {
                // lo <= base + code < hi, in code space, clamped to the codes that exist
                auto clampc = [&](int64_t x) { return x < 0 ? 0 : x > ncode ? ncode : x; };
                const bool lo_ok = !__builtin_sub_overflow(rlo, b.base, &clo);
                const bool hi_ok = !__builtin_sub_overflow(rhi, b.base, &chi);
                clo = lo_ok ? clampc(clo) : (rlo < 0 ? 0 : ncode);
                chi = hi_ok ? clampc(chi) : (rhi < 0 ? 0 : ncode);
            }
            b.code_lo = (uint32_t)std::min<int64_t>(clo, ncode - 1);
            b.code_span = (uint32_t)std::max<int64_t>(0, chi - clo);
            b.key_lo = (b.key >= 0 && P.keys[b.key].via_lut) ? slot_keys[b.key].front() : 0;
        }
        if (fast) {
            P.w0 = b.w;
            P.fast_big = big ? 1 : 0;
            if (big) lut16[0].clear();      // no code table
        }
    }

    // The generic row path tests a range (or no predicate) in registers, and
    // a key whose reachable values are contiguous is slot = key - key_lo, so
    // such columns drop their code table (up to 32 KB of LDS per workgroup,
    // which goes to the group table instead).
    if (!P.w0) {
        for (int s = 0; s < P.n_bp; ++s) {
            if (lut16[s].empty()) continue;
            BpCol& b = P.bp[s];
            const Fold& f = fold[bp_cols[s]];
            if (f.has_set || f.has_iv) continue;
            if (b.key >= 0) {
                const std::vector<int64_t>& sk = slot_keys[b.key];
                if (sk.back() - sk.front() + 1 != (int64_t)sk.size()) continue;
                b.key_lo = sk.front();
            }
            put_pred(f, b.pred, b.lo, b.hi, b.set, b.set_len);
            lut16[s].clear();
        }
    }

    // code tables.  Fast path: one byte per code holding the slot, G for a key
    // out of its domain, G + 1 for rejected codes, plus a reject entry at
    // index 2^w for rows the RLE predicates removed.  Otherwise uint8 (254 =
    // domain, 255 = reject) when the slots fit, else uint16.
    std::vector<bool> has_lut(P.n_bp, false);
    for (int s = 0; s < P.n_bp; ++s) {
        if (lut16[s].empty()) continue;
        BpCol& b = P.bp[s];
        const std::vector<uint16_t>& lut = lut16[s];
        const int64_t n = (int64_t)lut.size();
        has_lut[s] = true;
        if (P.w0 && s == 0) {
            std::vector<uint8_t> l8((n + 4 + 3) & ~int64_t(3), (uint8_t)(G + 1));
            for (int64_t code = 0; code < n; ++code)
                l8[code] = lut[code] == kLutReject ? (uint8_t)(G + 1) : lut[code] == kLutDomain ? (uint8_t)G
                                                                                           : (uint8_t)lut[code];
            b.lut_u8 = 1;
            b.lut_bytes = (int32_t)l8.size();
            b.ones_reject = l8[n - 1] == (uint8_t)(G + 1) ? 1 : 0;
            fix_ptr(&b.lut, blob_put(l8.data(), l8.size()));
            continue;
        }
        const bool u8 = b.key < 0 || P.keys[b.key].radix <= 254;
        b.lut_u8 = u8 ? 1 : 0;
        if (u8) {
            std::vector<uint8_t> l8((n + 3) & ~int64_t(3), 255);
            for (int64_t code = 0; code < n; ++code)
                l8[code] = lut[code] == kLutReject ? 255 : lut[code] == kLutDomain ? 254 : (uint8_t)lut[code];
            b.lut_bytes = (int32_t)l8.size();
            fix_ptr(&b.lut, blob_put(l8.data(), l8.size()));
        } else {
            std::vector<uint16_t> l16 = lut;
            if (l16.size() % 2) l16.push_back(kLutReject);
            b.lut_bytes = (int32_t)(l16.size() * 2);
            fix_ptr(&b.lut, blob_put(l16.data(), l16.size() * 2));
        }
    }

    // LDS layout: shared part (code tables, then the group tables) then kWaves slices
    size_t sh = 0;
    for (int s = 0; s < P.n_bp; ++s) {
        if (has_lut[s] && !P.w0) {       // the fast path keeps its table in static LDS
            P.bp[s].lut_lds_off = (int32_t)sh;
            sh = align16(sh + (size_t)P.bp[s].lut_bytes);
        }
        if (P.bp[s].or_bits_words > 0) {
            P.bp[s].or_bits_lds_off = (int32_t)sh;
            sh = align16(sh + 4 * (size_t)P.bp[s].or_bits_words);
        }
    }
    if (P.w0 && P.fast_big) {
        // one uint32 count per slot (G, G + 1: out of domain, rejected) in
        // dynamic LDS; Index sums go to the global table
        P.fast_rep_shift = 0;
        P.fast_sum_off = (int32_t)sh;
        sh = align16(sh + (size_t)(G + 2) * 4);
        P.fast_isum_off = -1;
        P.fast_bytes = (int32_t)(sh - P.fast_sum_off);
        P.table_lds = 0;
    } else if (P.w0) {
        // lane-replicated uint32 counts in static LDS: 32 replicas (a wave64 LDS
        // operation runs as two halves of 32 lanes, so no two lanes of a half
        // share an address), fewer when the slots do not fit
        const bool sum_bp = P.bp[0].sum_slot >= 0;
        int rs = 5;
        while (rs > 3 && ((G + 2) << rs) > kFastCntWords) --rs;
        P.fast_rep_shift = rs;
        P.fast_sum_off = (int32_t)sh;
        if (sum_bp) sh = align16(sh + ((size_t)G * 8 << rs));
        P.fast_isum_off = (int32_t)sh;
        sh = align16(sh + (size_t)P.n_idx * G * 8);
        P.fast_bytes = (int32_t)(sh - P.fast_sum_off);
        P.table_lds = 0;
    } else if (!P.row_mode) {
        // run mode adds once per group segment: int64 cells in LDS up to
        // kLdsTableBytes, else the global table
        const size_t table_bytes = sizeof(int64_t) * (size_t)(1 + P.n_sums) * (size_t)G;
        if (table_bytes <= (size_t)kLdsTableBytes) {
            P.table_lds = 1;
            P.table_lds_groups = G;
            P.table_lds_off = (int32_t)sh;
            sh = align16(sh + table_bytes);
        }
    } else {
        P.table_lds = 0;      // generic row path: placed below, once the wave slice is known
    }
    P.lds_shared_bytes = (int32_t)sh;

    // wave slice.  Fast row path: a 128-word toggle bitmap per RLE column (two
    // tiles are masked together; runs are never staged).  Otherwise a
    // 256-byte header (per-column staged counts, first runs and next-tile
    // cursors), then the staged runs, then row-mode buffers.
    size_t wv = 0;
    if (P.w0) {
        P.run_cap = 0;
        P.off_run_end = P.off_run_val = 0;
        P.off_tog = (int32_t)wv;
        wv = align16(wv + 512 * (size_t)std::max(P.k_rle, 1));
        P.off_pts = (int32_t)wv;
        P.lds_wave_bytes = (int32_t)wv;
        P.lds_dyn_bytes = (int32_t)(sh + kWaves * wv);
        if ((size_t)P.lds_dyn_bytes + kernel_static_lds(P.w0, P.fast_big) > t->ctx->lds_per_block)
            return fail(CCQ_E_UNSUPPORTED, "query needs %d bytes of LDS per workgroup (limit %zu)", P.lds_dyn_bytes,
                        t->ctx->lds_per_block);
        return CCQ_OK;
    }
    wv = 256;
    P.off_run_end = (int32_t)wv;
    wv = align16(wv + 4 * (size_t)P.run_cap);
    P.off_run_val = (int32_t)wv;
    wv = align16(wv + 8 * (size_t)P.run_cap);

    // run-boundary bitmaps and their word prefixes (one of each per RLE
    // column), a scratch toggle bitmap (when a column has predicates) and the
    // lanes' surviving-row words (when Index points are read)
    P.off_bnd = (int32_t)wv;
    wv = align16(wv + 256 * (size_t)std::max(P.k_rle, 1));
    P.off_bpre = (int32_t)wv;
    wv = align16(wv + 256 * (size_t)std::max(P.k_rle, 1));
    bool any_pred = false;
    for (int s = 0; s < P.k_rle; ++s) any_pred = any_pred || P.rle[s].pred != kPredNone;
    any_pred = any_pred || idx_pred;     // Index predicates use the same scratch bitmap
    P.off_tog = any_pred ? (int32_t)wv : -1;
    if (any_pred) wv = align16(wv + 256);
    P.off_pmw = (int32_t)wv;
    if (P.n_idx > 0) wv = align16(wv + 256);
    P.off_rcl = row_clause ? (int32_t)wv : -1;
    if (row_clause) wv = align16(wv + 256);
    // run mode with a global group table: LDS slots merging group segments
    P.seg_slots = (!P.row_mode && P.n_keys > 0 && !P.table_lds) ? 1 : 0;
    P.off_slots = (int32_t)wv;
    if (P.seg_slots) wv = align16(wv + (size_t)kSegSlots * (2 + P.n_sums) * 8);
    if (P.row_mode) {
        // generic row mode: the staged packed words of the tile
        for (int s = 0; s < P.n_bp; ++s) {
            P.bp[s].stage_off = (int32_t)wv;
            wv = align16(wv + 4 * (size_t)(64 * P.bp[s].w + 2));
        }
        // composite columns: the tile's listed rows (one word per lane) and
        // the exclusive prefix of their popcounts
        for (int i = 0; i < P.n_comp; ++i) {
            P.comp[i].lds_off = (int32_t)wv;
            wv = align16(wv + 2 * 256);
        }
    }
    P.off_pts = 0;
    P.lds_wave_bytes = (int32_t)wv;

    // The generic row path's group table, per workgroup in LDS, added to
    // the global table once at the end.  A bit-packed key changes from row
    // to row, so the table takes compact 32-bit cells, as many groups as the
    // workgroup's LDS allows, while a workgroup counts fewer than 2^31 rows
    // (the counts are uint32).
    if (P.row_mode) {
        // Groups [0, table_lds_groups) get LDS cells, the rest add to the
        // global table.  With a bit-packed key the group changes from row to
        // row, so the table takes what LDS is left; with RLE keys only, rows
        // reach the table about once per run, and a table beyond
        // kLdsTableBytes stays global (keeping occupancy).
        bool bp_keyed = false;
        for (int k = 0; k < P.n_keys; ++k) bp_keyed = bp_keyed || P.keys[k].src_kind == kKeyBp;
        // LDS columns: COUNT and the SUMs added per row; an Index SUM (a few
        // points per tile) adds to the global table directly
        uint64_t map = 0;
        int cols = 0;
        for (int w = 0; w <= P.n_sums; ++w) {
            bool idx_sum = false;
            for (int j = 0; j < P.n_idx; ++j) idx_sum = idx_sum || (w > 0 && P.idx[j].sum_slot == w - 1);
            // MIN and MAX keep 64-bit encoded values: the global table, through the registers
            const bool minmax = w > 0 && w - 1 < P.n_ext && P.ext[w - 1].kind != kExtSum;
            map |= (uint64_t)((idx_sum || minmax) ? 15 : cols++) << (4 * w);
        }
        const size_t cell_row = sizeof(uint32_t) * (size_t)cols;
        const int64_t min_blocks = std::max<int64_t>(1, std::min<int64_t>((P.n_tiles + 3) / 4, t->ctx->cus));
        const int64_t rows_per_wg = ((P.n_tiles + 4 * min_blocks - 1) / (4 * min_blocks)) * 4 * P.tile_rows;
        // dynamic LDS left: the workgroup's LDS minus the kernel's static LDS
        const size_t avail = t->ctx->lds_per_block - (size_t)kernel_static_lds(0, 0);
        const size_t used = align16(sh) + kWaves * wv;
        int64_t lg = 0;
        if (used < avail) lg = (int64_t)((avail - used) / cell_row) & ~int64_t(3);
        lg = std::min<int64_t>(lg, G);
        // Occupancy before coverage: when a bit-packed key's table would keep
        // the workgroup alone on its CU, the table keeps only as many groups
        // as let two workgroups share the CU (if that is at least
        // kLdsShareMin), and the groups above add to the global table.  (In
        // a batch, one such plan left whole would hold its whole launch to
        // one workgroup per CU.)
        // Results do not change.  Dictionary codes numbered
        // by frequency keep their hot groups in LDS (measured: the c4 batch
        // 355 -> 235 ms); with codes in random order about half the rows
        // would add to the global table, about as fast as one workgroup per CU.
        const size_t avail2 = t->ctx->lds_per_block / 2 - (size_t)kernel_static_lds(0, 0);
        const int64_t lg2 = avail2 > used ? (int64_t)((avail2 - used) / cell_row) & ~int64_t(3) : 0;
        if (bp_keyed && lg > kLdsShareGroups && lg2 >= kLdsShareMin) lg = std::min<int64_t>(lg, lg2);
        if (!bp_keyed && (size_t)G * cell_row > (size_t)kLdsTableBytes) lg = 0;
        if (lg > 0 && rows_per_wg < ((int64_t)1 << 31)) {
            P.table_lds = 1;
            P.table_c32 = 1;
            P.table_lds_groups = lg;
            P.table_lds_map = map;
            P.table_lds_cols = cols;
            P.table_lds_off = (int32_t)sh;
            sh = align16(sh + (size_t)lg * cell_row);
        }
    }
    P.lds_shared_bytes = (int32_t)sh;
    P.lds_dyn_bytes = (int32_t)(sh + kWaves * wv);
    if ((size_t)P.lds_dyn_bytes + kernel_static_lds(P.w0, P.fast_big) > t->ctx->lds_per_block)
        return fail(CCQ_E_UNSUPPORTED, "query needs %d bytes of LDS per workgroup (limit %zu)", P.lds_dyn_bytes,
                    t->ctx->lds_per_block);

    return CCQ_OK;
}

}  // namespace

extern "C" {

ccq_status ccq_plan_check(const ccq_table* t, const ccq_query_desc* q, int64_t* max_groups,
                          size_t* workspace_bytes) {
    Compiled c;
    if (ccq_status s = compile_plan(t, q, c)) return s;
    if (max_groups) *max_groups = c.P.n_keys == 0 ? 1 : c.P.n_groups;
    if (workspace_bytes) *workspace_bytes = workspace_layout(c.P).total;
    return ok();
}

ccq_status ccq_plan_create(const ccq_table* t, const ccq_query_desc* q, ccq_plan** out) {
    if (!out) return fail(CCQ_E_INVALID, "out is NULL");
    *out = nullptr;
    Compiled c;
    if (ccq_status s = compile_plan(t, q, c)) return s;
    if (t->ctx->device < 0) return fail(CCQ_E_UNSUPPORTED, "host-only context: plans can be checked, not created");
    DevPlan& P = c.P;
    hipError_t e = hipSetDevice(t->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    void* dblob = nullptr;
    e = hipMalloc(&dblob, c.blob.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(plan)");
    for (const auto& f : c.fixes) {
        const uint64_t addr = (uint64_t)((unsigned char*)dblob + f.second);
        memcpy((unsigned char*)&P + f.first, &addr, sizeof addr);
    }
    memcpy(c.blob.data(), &P, sizeof P);
    e = hipMemcpy(dblob, c.blob.data(), c.blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dblob);
        return hip_fail(e, "hipMemcpy(plan)");
    }
    ccq_plan* p = new (std::nothrow) ccq_plan;
    if (!p) {
        (void)hipFree(dblob);
        return fail(CCQ_E_NOMEM, "out of host memory");
    }
    p->ctx = t->ctx;
    p->host = P;
    p->dev = (DevPlan*)dblob;
    p->blob = dblob;
    p->grid_fused = fused_grid_limit(P, t->ctx->cus);
    p->max_groups = P.n_keys == 0 ? 1 : P.n_groups;
    p->ws = workspace_layout(P);
    *out = p;
    return ok();
}

void ccq_plan_destroy(ccq_plan* p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    (void)hipFree(p->blob);
    delete p;
}

ccq_status ccq_plan_info(const ccq_plan* p, int64_t* max_groups, size_t* workspace_bytes) {
    if (!p) return fail(CCQ_E_INVALID, "plan is NULL");
    if (max_groups) *max_groups = p->max_groups;
    if (workspace_bytes) *workspace_bytes = p->ws.total;
    return ok();
}

ccq_status ccq_execute(const ccq_plan* p, void* workspace, size_t workspace_bytes, void* stream,
                       const ccq_result* r) {
    return ccq_execute_ex(p, workspace, workspace_bytes, stream, r, nullptr);
}

namespace {

// checks shared by the execute entry points (workspace checked by the caller)
ccq_status check_result(const ccq_plan* p, const ccq_result* r) {
    if (r->capacity < p->max_groups)
        return fail(CCQ_E_CAPACITY, "result capacity %lld < max groups %lld", (long long)r->capacity,
                    (long long)p->max_groups);
    if (!r->counts || !r->n_groups || !r->status || (p->host.n_keys && !r->keys) || (p->host.n_aggs && !r->aggs))
        return fail(CCQ_E_INVALID, "result buffers missing");
    return CCQ_OK;
}

}  // namespace

ccq_status ccq_execute_ex(const ccq_plan* p, void* workspace, size_t workspace_bytes, void* stream,
                          const ccq_result* r, const ccq_exec_opts* opts) {
    if (!p || !r) return fail(CCQ_E_INVALID, "plan or result is NULL");
    if (!workspace || ((uintptr_t)workspace & 255)) return fail(CCQ_E_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes < p->ws.total)
        return fail(CCQ_E_CAPACITY, "workspace of %zu bytes, plan needs %zu", workspace_bytes, p->ws.total);
    if (ccq_status s = check_result(p, r)) return s;
    hipError_t e = hipSetDevice(p->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = launch_query(p->host, p->dev, workspace, (hipStream_t)stream, r->keys, r->counts, r->aggs, r->n_groups,
                     r->status, p->grid_fused, opts ? (hipEvent_t)opts->fused_begin : nullptr,
                     opts ? (hipEvent_t)opts->fused_end : nullptr);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return ok();
}

ccq_status ccq_execute_noalloc(const ccq_plan* p, void* stream, const ccq_result* r) {
    if (!p || !r) return fail(CCQ_E_INVALID, "plan or result is NULL");
    if (p->ws.total > kScratchBytes)
        return fail(CCQ_E_CAPACITY, "plan needs a %zu-byte workspace; the fixed scratch holds %zu", p->ws.total,
                    kScratchBytes);
    if (!p->ctx->scratch) return fail(CCQ_E_INVALID, "context has no device scratch");
    if (ccq_status s = check_result(p, r)) return s;
    hipError_t e = hipSetDevice(p->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    // the launch sequence clears the status header and the group table itself
    e = launch_query(p->host, p->dev, p->ctx->scratch, (hipStream_t)stream, r->keys, r->counts, r->aggs,
                     r->n_groups, r->status, p->grid_fused, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return ok();
}

}  // extern "C"

static_assert(ccq::kScratchBytes == CCQ_NOALLOC_WORKSPACE_BYTES, "fixed scratch size differs from the header's");

static_assert(kOpNone == CCQ_OP_NONE && kOpAdd == CCQ_OP_ADD && kOpSub == CCQ_OP_SUB && kOpMul == CCQ_OP_MUL,
              "ExtOp values follow the ABI");

extern "C" ccq_status ccq_avg_var(const int64_t* count, const int64_t* sum, const int64_t* sum_sq, int64_t n_rows,
                                  double* avg, double* var) {
    if (n_rows < 0 || (n_rows > 0 && (!count || !sum || !sum_sq || !avg || !var)))
        return ccq::fail(CCQ_E_INVALID, "bad arguments");
    for (int64_t i = 0; i < n_rows; ++i) {
        if (count[i] == 0) {
            avg[i] = var[i] = 0.0;
            continue;
        }
        // each exact integer rounded once, then the formula in this order
        const volatile double n = (double)count[i], s = (double)sum[i], ss = (double)sum_sq[i];
        const volatile double a = s / n;
        const volatile double sq = s * s;
        const volatile double m = sq / n;
        const volatile double d = ss - m;
        avg[i] = a;
        var[i] = d / n;
    }
    return ccq::ok();
}
