/*
 * ccq_oracle -- plain CPU reference for filter / group-by / aggregate queries
 * over lightweight-encoded columns.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg load this library.  The GPU library shares no code,
 * header, table or helper with it.
 *
 * What it computes is the plain relational definition (the paper's method is
 * exact, so its answer must equal the uncompressed one):
 *   1. every referenced column is decompressed to one int64 value per logical
 *      row (Section 3.1 "Basic Encodings": RLE runs (value, start, end), Index
 *      (value, position); Section 3.2 bit-width reduction with a global
 *      reference value, value = base + code; Section 3.2 composite encodings:
 *      RLE + Index is pure runs (value, start, end) and Index points on the
 *      rows no run covers, disjoint and together covering every row; Plain +
 *      Index is the bit-packed codes with the outlier rows listed as Index
 *      points, whose codes are never read);
 *   2. a row qualifies when every clause holds on its values (selection,
 *      Section 6): a clause is one predicate, or the OR of the predicates
 *      that share a clause id (OR, Section 5.2); a negated predicate holds
 *      where the plain one fails (NOT, Section 5.3);
 *   3. qualifying rows are grouped by their key tuple and COUNT(*), SUM, MIN
 *      and MAX are accumulated per group (Section 7, grouping and aggregating
 *      phases); an aggregate's argument is a column or the row-wise sum,
 *      difference or product of two columns (Section 6, arithmetic on
 *      aligned columns);
 *   4. groups are emitted in ascending key order (torch.unique returns sorted
 *      unique values, Section 2.2); an ungrouped query emits one row.
 * No NULLs exist (Appendix "Query Optimization Rules").
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - run ends are stored exclusive: run i covers rows [run_ends[i-1], run_ends[i]),
 *     i.e. the paper's inclusive end plus one; base columns have no gaps;
 *   - an Index data column holds 0 at rows it does not list;
 *   - range predicates are half open, lo <= v < hi; IN has set semantics;
 *   - a group key is v >> shift and must lie in the declared [0, card);
 *   - the bit-packed stream is LSB first in little-endian uint32 words;
 *   - sums, differences and products are exact int64; any overflow is
 *     reported as an error;
 *   - an ungrouped query over no qualifying row reports 0 for every
 *     aggregate (MIN and MAX included).
 *
 * Work is split into chunks of at most 2^20 rows handed to std::threads; each
 * thread keeps its own std::map, and the maps are added together at the end
 * (exact integer addition, so the thread count cannot change the answer).
 */
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

extern "C" {

enum { ORC_RLE = 1, ORC_INDEX = 2, ORC_BITPACKED = 3, ORC_RLE_INDEX = 4, ORC_PLAIN_INDEX = 5 };
enum { ORC_I32 = 1, ORC_I64 = 2 };
enum { ORC_RANGE = 1, ORC_IN = 2, ORC_NOT_RANGE = 3, ORC_NOT_IN = 4 };
enum { ORC_COUNT = 1, ORC_SUM = 2, ORC_MIN = 3, ORC_MAX = 4 };
enum { ORC_OP_NONE = 0, ORC_OP_ADD = 1, ORC_OP_SUB = 2, ORC_OP_MUL = 3 };

typedef struct {
    int32_t enc;
    int32_t vtype;
    int64_t n;                  /* runs | listed points | rows */
    const void* values;         /* RLE / INDEX values */
    const int64_t* run_ends;    /* RLE */
    const void* positions;      /* INDEX, int32 or int64 per ptype */
    const uint32_t* packed;     /* BITPACKED */
    int32_t w;                  /* BITPACKED bit width */
    int32_t ptype;              /* INDEX position type: ORC_I32 or ORC_I64 */
    int64_t base;               /* BITPACKED: value = base + code */
    /* composite encodings (Section 3.2) */
    const int64_t* run_starts;  /* RLE_INDEX: first row of each pure run (its end exclusive in run_ends) */
    int64_t pt_n;               /* RLE_INDEX, PLAIN_INDEX: listed points */
    const void* pt_positions;   /* strictly increasing, pt_ptype */
    const void* pt_values;      /* pt_vtype */
    int32_t pt_ptype, pt_vtype;
} orc_column;

typedef struct {
    int32_t col;
    int32_t op;
    int64_t lo, hi;             /* RANGE: lo <= v < hi */
    const int64_t* in_list;     /* IN */
                                /* NOT_RANGE, NOT_IN: the negations (Section 5.3) */
    int64_t in_len;
    int32_t clause;             /* 0: a clause of its own; k > 0: ORed with the others of clause k */
    int32_t pad_;
} orc_pred;

typedef struct {
    int32_t col;
    int32_t shift;
    int64_t card;
} orc_key;

typedef struct {
    int32_t func;
    int32_t col;
    int32_t op;     /* ORC_OP_NONE: the column; else col op col2, row by row */
    int32_t col2;
} orc_agg;

}  // extern "C"

namespace {

struct Acc {
    int64_t count = 0;
    std::vector<int64_t> vals;
};

struct Result {
    std::string error;
    int32_t n_keys = 0, n_aggs = 0;
    std::vector<std::vector<int64_t>> keys;
    std::vector<int64_t> counts;
    std::vector<std::vector<int64_t>> aggs;
};

int64_t value_at(const orc_column& c, int64_t i) {
    return c.vtype == ORC_I32 ? (int64_t)((const int32_t*)c.values)[i] : ((const int64_t*)c.values)[i];
}

int64_t position_at(const orc_column& c, int64_t i) {
    return c.ptype == ORC_I32 ? (int64_t)((const int32_t*)c.positions)[i] : ((const int64_t*)c.positions)[i];
}

int64_t point_position(const orc_column& c, int64_t i) {
    return c.pt_ptype == ORC_I32 ? (int64_t)((const int32_t*)c.pt_positions)[i]
                                 : ((const int64_t*)c.pt_positions)[i];
}

int64_t point_value(const orc_column& c, int64_t i) {
    return c.pt_vtype == ORC_I32 ? (int64_t)((const int32_t*)c.pt_values)[i] : ((const int64_t*)c.pt_values)[i];
}

/* first point of a composite column whose position is >= r */
int64_t first_composite_point(const orc_column& c, int64_t r) {
    int64_t lo = 0, hi = c.pt_n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (point_position(c, mid) < r) lo = mid + 1; else hi = mid;
    }
    return lo;
}

std::string validate_points(const orc_column& c, int64_t n_rows) {
    if (c.pt_ptype != ORC_I32 && c.pt_ptype != ORC_I64) return "point position type must be int32 or int64";
    if (c.pt_vtype != ORC_I32 && c.pt_vtype != ORC_I64) return "point value type must be int32 or int64";
    if (c.pt_n < 0 || (c.pt_n > 0 && (!c.pt_positions || !c.pt_values))) return "point arrays missing";
    int64_t prev = -1;
    for (int64_t i = 0; i < c.pt_n; i++) {
        int64_t p = point_position(c, i);
        if (p <= prev || p >= n_rows) return "point positions must be strictly increasing in [0, rows)";
        prev = p;
    }
    return "";
}

/* first listed point whose position is >= r (binary search over positions) */
int64_t first_point_at_or_after(const orc_column& c, int64_t r) {
    int64_t lo = 0, hi = c.n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (position_at(c, mid) < r) lo = mid + 1; else hi = mid;
    }
    return lo;
}

std::string validate_column(const orc_column& c, int64_t n_rows) {
    if (c.enc == ORC_RLE) {
        if (c.vtype != ORC_I32 && c.vtype != ORC_I64) return "RLE value type must be int32 or int64";
        if (c.n <= 0 || !c.run_ends || !c.values) return "RLE column needs at least one run";
        int64_t prev = 0;
        for (int64_t i = 0; i < c.n; i++) {
            if (c.run_ends[i] <= prev) return "RLE run ends must be strictly increasing and positive";
            prev = c.run_ends[i];
        }
        if (prev != n_rows) return "last RLE run end must equal the row count";
    } else if (c.enc == ORC_INDEX) {
        if (c.vtype != ORC_I32 && c.vtype != ORC_I64) return "Index value type must be int32 or int64";
        if (c.ptype != ORC_I32 && c.ptype != ORC_I64) return "Index position type must be int32 or int64";
        if (c.n < 0 || (c.n > 0 && (!c.positions || !c.values))) return "Index column arrays missing";
        int64_t prev = -1;
        for (int64_t i = 0; i < c.n; i++) {
            int64_t p = position_at(c, i);
            if (p <= prev || p >= n_rows) return "Index positions must be strictly increasing in [0, rows)";
            prev = p;
        }
    } else if (c.enc == ORC_BITPACKED || c.enc == ORC_PLAIN_INDEX) {
        if (c.w < 1 || c.w > 32) return "bit width must be in 1..32";
        if (!c.packed) return "packed stream missing";
        if (c.n != n_rows) return "bit-packed column must hold one code per row";
        if (c.enc == ORC_PLAIN_INDEX) return validate_points(c, n_rows);
    } else if (c.enc == ORC_RLE_INDEX) {
        if (c.vtype != ORC_I32 && c.vtype != ORC_I64) return "RLE value type must be int32 or int64";
        if (c.n < 0 || (c.n > 0 && (!c.values || !c.run_starts || !c.run_ends))) return "RLE part arrays missing";
        std::string e = validate_points(c, n_rows);
        if (!e.empty()) return e;
        /* pure runs in order, disjoint; points on none of them; together every row */
        int64_t prev_end = 0, covered = 0;
        for (int64_t i = 0; i < c.n; i++) {
            if (c.run_starts[i] < prev_end || c.run_ends[i] <= c.run_starts[i] || c.run_ends[i] > n_rows)
                return "RLE part runs must be non-empty, ordered, disjoint and inside the rows";
            covered += c.run_ends[i] - c.run_starts[i];
            prev_end = c.run_ends[i];
        }
        for (int64_t k = 0; k < c.pt_n; k++) {
            int64_t p = point_position(c, k);
            int64_t i = std::upper_bound(c.run_ends, c.run_ends + c.n, p) - c.run_ends;
            if (i < c.n && c.run_starts[i] <= p) return "a point lies inside a pure run";
        }
        if (covered + c.pt_n != n_rows) return "runs and points must cover every row";
    } else {
        return "unknown encoding";
    }
    return "";
}

/* Rows [r0, r1) of column c as int64 values. */
void decode(const orc_column& c, int64_t r0, int64_t r1, int64_t* out) {
    int64_t len = r1 - r0;
    if (len <= 0) return;
    if (c.enc == ORC_RLE) {
        /* first run whose (exclusive) end lies beyond r0 is the run holding row r0 */
        int64_t i = std::upper_bound(c.run_ends, c.run_ends + c.n, r0) - c.run_ends;
        int64_t r = r0;
        while (r < r1) {
            int64_t stop = std::min(c.run_ends[i], r1);
            int64_t v = value_at(c, i);
            for (; r < stop; r++) out[r - r0] = v;
            i++;
        }
    } else if (c.enc == ORC_INDEX) {
        for (int64_t k = 0; k < len; k++) out[k] = 0;
        for (int64_t i = first_point_at_or_after(c, r0); i < c.n && position_at(c, i) < r1; i++)
            out[position_at(c, i) - r0] = value_at(c, i);
    } else if (c.enc == ORC_RLE_INDEX) {
        /* pure runs first (rows between them are points, filled below) */
        for (int64_t i = std::upper_bound(c.run_ends, c.run_ends + c.n, r0) - c.run_ends;
             i < c.n && c.run_starts[i] < r1; i++) {
            int64_t v = value_at(c, i);
            for (int64_t r = std::max(c.run_starts[i], r0); r < std::min(c.run_ends[i], r1); r++) out[r - r0] = v;
        }
    } else {
        const uint64_t mask = c.w == 32 ? 0xFFFFFFFFull : ((1ull << c.w) - 1);
        for (int64_t r = r0; r < r1; r++) {
            uint64_t bit = (uint64_t)r * (uint64_t)c.w;
            uint64_t word = bit / 32, sh = bit % 32;
            uint64_t two = (uint64_t)c.packed[word] | ((uint64_t)c.packed[word + 1] << 32);
            uint64_t code = (two >> sh) & mask;
            out[r - r0] = c.base + (int64_t)code;
        }
    }
    /* composite: the Index part's rows take the points' values */
    if (c.enc == ORC_RLE_INDEX || c.enc == ORC_PLAIN_INDEX)
        for (int64_t i = first_composite_point(c, r0); i < c.pt_n && point_position(c, i) < r1; i++)
            out[point_position(c, i) - r0] = point_value(c, i);
}

struct Query {
    std::vector<orc_column> cols;
    int64_t n_rows = 0;
    std::vector<orc_pred> preds;
    std::vector<std::set<int64_t>> in_sets;
    std::vector<std::vector<size_t>> clauses;   /* predicate indices per clause; a row needs one of each */
    std::vector<orc_key> keys;
    std::vector<orc_agg> aggs;
    int64_t row_begin = 0, row_end = 0;
    std::vector<int> used;        /* referenced column ids */
    std::vector<int> slot;        /* column id -> index into the decoded chunk */
};

std::vector<int64_t> initial_vals(const Query& q) {
    std::vector<int64_t> v(q.aggs.size(), 0);
    for (size_t a = 0; a < q.aggs.size(); a++) {
        if (q.aggs[a].func == ORC_MIN) v[a] = INT64_MAX;
        if (q.aggs[a].func == ORC_MAX) v[a] = INT64_MIN;
    }
    return v;
}

/* fold x into accumulator v of aggregate a; false on overflow */
bool fold(const orc_agg& a, int64_t& v, int64_t x) {
    if (a.func == ORC_MIN) v = std::min(v, x);
    else if (a.func == ORC_MAX) v = std::max(v, x);
    else return !__builtin_add_overflow(v, x, &v);
    return true;
}

struct ThreadState {
    std::map<std::vector<int64_t>, Acc> groups;
    std::string error;
};

void run_chunks(const Query& q, std::atomic<int64_t>& next_chunk, int64_t n_chunks, ThreadState& st) {
    const int64_t CH = 1 << 20;
    std::vector<std::vector<int64_t>> x(q.used.size());
    std::vector<int64_t> key(q.keys.size());
    std::vector<int64_t> last_key;
    Acc* last = nullptr;
    for (;;) {
        int64_t ch = next_chunk.fetch_add(1);
        if (ch >= n_chunks || !st.error.empty()) return;
        int64_t c0 = q.row_begin + ch * CH;
        int64_t c1 = std::min(c0 + CH, q.row_end);
        for (size_t u = 0; u < q.used.size(); u++) {
            x[u].resize(c1 - c0);
            decode(q.cols[q.used[u]], c0, c1, x[u].data());
        }
        for (int64_t r = 0; r < c1 - c0; r++) {
            auto holds = [&](size_t p) {
                const int64_t v = x[q.slot[q.preds[p].col]][r];
                const int32_t op = q.preds[p].op;
                bool h;
                if (op == ORC_RANGE || op == ORC_NOT_RANGE) h = q.preds[p].lo <= v && v < q.preds[p].hi;
                else h = q.in_sets[p].count(v) != 0;
                return (op == ORC_NOT_RANGE || op == ORC_NOT_IN) ? !h : h;
            };
            bool pass = true;
            for (size_t c = 0; c < q.clauses.size() && pass; c++) {
                bool any = false;
                for (size_t p : q.clauses[c]) any = any || holds(p);
                pass = any;
            }
            if (!pass) continue;
            for (size_t k = 0; k < q.keys.size(); k++) {
                int64_t v = x[q.slot[q.keys[k].col]][r] >> q.keys[k].shift;
                if (v < 0 || v >= q.keys[k].card) {
                    st.error = "group key outside its declared domain";
                    return;
                }
                key[k] = v;
            }
            if (last == nullptr || key != last_key) {
                auto it = st.groups.find(key);
                if (it == st.groups.end()) {
                    Acc a;
                    a.vals = initial_vals(q);
                    it = st.groups.emplace(key, a).first;
                }
                last = &it->second;
                last_key = key;
            }
            last->count += 1;
            for (size_t a = 0; a < q.aggs.size(); a++) {
                const orc_agg& ag = q.aggs[a];
                int64_t v = 1;
                bool ok = true;
                if (ag.func != ORC_COUNT) {
                    v = x[q.slot[ag.col]][r];
                    if (ag.op != ORC_OP_NONE) {
                        const int64_t w = x[q.slot[ag.col2]][r];
                        if (ag.op == ORC_OP_ADD) ok = !__builtin_add_overflow(v, w, &v);
                        else if (ag.op == ORC_OP_SUB) ok = !__builtin_sub_overflow(v, w, &v);
                        else ok = !__builtin_mul_overflow(v, w, &v);
                    }
                }
                if (!ok || !fold(ag, last->vals[a], v)) {
                    st.error = "int64 overflow in an aggregate";
                    return;
                }
            }
        }
    }
}

Result* execute(Query& q, int n_threads) {
    Result* res = new Result();
    res->n_keys = (int32_t)q.keys.size();
    res->n_aggs = (int32_t)q.aggs.size();
    for (auto& c : q.cols) {
        std::string e = validate_column(c, q.n_rows);
        if (!e.empty()) { res->error = e; return res; }
    }
    if (q.row_begin < 0 || q.row_end > q.n_rows || q.row_begin > q.row_end) {
        res->error = "window outside the table";
        return res;
    }
    q.slot.assign(q.cols.size(), -1);
    auto use = [&](int c) -> bool {
        if (c < 0 || c >= (int)q.cols.size()) return false;
        if (q.slot[c] < 0) { q.slot[c] = (int)q.used.size(); q.used.push_back(c); }
        return true;
    };
    q.in_sets.assign(q.preds.size(), {});
    std::map<int32_t, size_t> clause_at;
    for (size_t p = 0; p < q.preds.size(); p++) {
        if (!use(q.preds[p].col)) { res->error = "predicate column out of range"; return res; }
        const int32_t k = q.preds[p].clause;
        if (k < 0) { res->error = "negative clause id"; return res; }
        if (k == 0 || !clause_at.count(k)) {
            if (k != 0) clause_at[k] = q.clauses.size();
            q.clauses.push_back({});
        }
        q.clauses[k == 0 ? q.clauses.size() - 1 : clause_at[k]].push_back(p);
        if (q.preds[p].op == ORC_IN || q.preds[p].op == ORC_NOT_IN) {
            for (int64_t i = 0; i < q.preds[p].in_len; i++) q.in_sets[p].insert(q.preds[p].in_list[i]);
        } else if (q.preds[p].op != ORC_RANGE && q.preds[p].op != ORC_NOT_RANGE) {
            res->error = "unknown predicate";
            return res;
        }
    }
    for (auto& k : q.keys) {
        if (!use(k.col)) { res->error = "key column out of range"; return res; }
        if (k.card <= 0 || k.shift < 0 || k.shift > 62) { res->error = "bad key domain"; return res; }
    }
    for (auto& a : q.aggs) {
        if (a.func == ORC_SUM || a.func == ORC_MIN || a.func == ORC_MAX) {
            if (!use(a.col)) { res->error = "aggregate column out of range"; return res; }
            if (a.op < ORC_OP_NONE || a.op > ORC_OP_MUL) { res->error = "unknown operator"; return res; }
            if (a.op != ORC_OP_NONE && !use(a.col2)) { res->error = "aggregate column out of range"; return res; }
        } else if (a.func != ORC_COUNT) {
            res->error = "unknown aggregate";
            return res;
        }
    }

    const int64_t CH = 1 << 20;
    int64_t n_chunks = (q.row_end - q.row_begin + CH - 1) / CH;
    if (n_threads < 1) n_threads = 1;
    std::vector<ThreadState> st(n_threads);
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < n_threads; t++) th.emplace_back(run_chunks, std::cref(q), std::ref(next), n_chunks, std::ref(st[t]));
    for (auto& t : th) t.join();

    std::map<std::vector<int64_t>, Acc> all;
    for (auto& s : st) {
        if (!s.error.empty()) { res->error = s.error; return res; }
        for (auto& kv : s.groups) {
            auto it = all.find(kv.first);
            if (it == all.end()) { all.emplace(kv.first, kv.second); continue; }
            it->second.count += kv.second.count;
            for (size_t a = 0; a < q.aggs.size(); a++)
                if (!fold(q.aggs[a], it->second.vals[a], kv.second.vals[a])) {
                    res->error = "int64 overflow in an aggregate";
                    return res;
                }
        }
    }
    if (q.keys.empty()) {
        /* ungrouped: exactly one row, zero when nothing qualifies */
        Acc a;
        a.vals.assign(q.aggs.size(), 0);
        auto it = all.find(std::vector<int64_t>{});
        if (it != all.end() && it->second.count > 0) a = it->second;
        res->keys.push_back({});
        res->counts.push_back(a.count);
        res->aggs.push_back(a.vals);
        return res;
    }
    for (auto& kv : all) {   /* std::map iterates in ascending lexicographic key order */
        res->keys.push_back(kv.first);
        res->counts.push_back(kv.second.count);
        res->aggs.push_back(kv.second.vals);
    }
    return res;
}

}  // namespace

extern "C" {

/* Run one query; always returns a handle (check orc_error). */
void* orc_query(const orc_column* cols, int32_t n_cols, int64_t n_rows, const orc_pred* preds, int32_t n_preds,
                const orc_key* keys, int32_t n_keys, const orc_agg* aggs, int32_t n_aggs, int64_t row_begin,
                int64_t row_end, int32_t n_threads) {
    Query q;
    q.cols.assign(cols, cols + n_cols);
    q.n_rows = n_rows;
    q.preds.assign(preds, preds + n_preds);
    q.keys.assign(keys, keys + n_keys);
    q.aggs.assign(aggs, aggs + n_aggs);
    q.row_begin = row_begin;
    q.row_end = row_end;
    return execute(q, n_threads);
}

const char* orc_error(void* h) { return ((Result*)h)->error.c_str(); }

int64_t orc_n_groups(void* h) { return (int64_t)((Result*)h)->counts.size(); }

/* keys: [G][n_keys], counts: [G], aggs: [G][n_aggs] */
void orc_copy(void* h, int64_t* keys, int64_t* counts, int64_t* aggs) {
    Result* r = (Result*)h;
    for (size_t g = 0; g < r->counts.size(); g++) {
        for (int k = 0; k < r->n_keys; k++) keys[g * r->n_keys + k] = r->keys[g][k];
        counts[g] = r->counts[g];
        for (int a = 0; a < r->n_aggs; a++) aggs[g * r->n_aggs + a] = r->aggs[g][a];
    }
}

void orc_free(void* h) { delete (Result*)h; }

/* Decode rows [r0, r1) of one column; returns "" or a validation message. */
const char* orc_decode(const orc_column* c, int64_t n_rows, int64_t r0, int64_t r1, int64_t* out) {
    static thread_local std::string err;
    err = validate_column(*c, n_rows);
    if (!err.empty()) return err.c_str();
    if (r0 < 0 || r1 > n_rows || r0 > r1) { err = "rows outside the column"; return err.c_str(); }
    decode(*c, r0, r1, out);
    return "";
}

}  // extern "C"
