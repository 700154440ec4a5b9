// Standalone driver for the CPU oracle under AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure; built and run by
// tests/test_oracle_sanitize.py with g++ on the host only).
//
// It links oracle/ccq_oracle.cpp directly, builds seeded random tables (RLE
// with int32 and int64 values, Index with int32 and int64 positions,
// bit-packed columns of every width, RLE + Index and Plain + Index
// composites), runs queries with range / IN / NOT
// predicates, OR clauses, keys, SUM / MIN / MAX and two-column expressions
// over several thread counts and windows, and checks every answer against
// its own row-by-row evaluation.  Any sanitizer report aborts the process.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <random>
#include <vector>

extern "C" {
typedef struct {
    int32_t enc, vtype;
    int64_t n;
    const void* values;
    const int64_t* run_ends;
    const void* positions;
    const uint32_t* packed;
    int32_t w, ptype;
    int64_t base;
    const int64_t* run_starts;
    int64_t pt_n;
    const void* pt_positions;
    const void* pt_values;
    int32_t pt_ptype, pt_vtype;
} orc_column;
typedef struct {
    int32_t col, op;
    int64_t lo, hi;
    const int64_t* in_list;
    int64_t in_len;
    int32_t clause, pad_;
} orc_pred;
typedef struct {
    int32_t col, shift;
    int64_t card;
} orc_key;
typedef struct {
    int32_t func, col, op, col2;
} orc_agg;
void* orc_query(const orc_column*, int32_t, int64_t, const orc_pred*, int32_t, const orc_key*, int32_t,
                const orc_agg*, int32_t, int64_t, int64_t, int32_t);
const char* orc_error(void*);
int64_t orc_n_groups(void*);
void orc_copy(void*, int64_t*, int64_t*, int64_t*);
void orc_free(void*);
}

namespace {

std::mt19937_64 rng(12345);
int64_t uni(int64_t lo, int64_t hi) { return lo + (int64_t)(rng() % (uint64_t)(hi - lo)); }

struct Col {
    orc_column d{};
    std::vector<int32_t> v32, p32;
    std::vector<int64_t> v64, ends, p64, starts, pv;
    std::vector<uint32_t> packed;
    std::vector<int64_t> rows;   // the decoded column, for the driver's own evaluation
};

Col make_rle(int64_t n, bool wide) {
    Col c;
    int64_t r = 0;
    while (r < n) {
        r = std::min(n, r + uni(1, 9));
        c.ends.push_back(r);
    }
    for (size_t i = 0; i < c.ends.size(); ++i) {
        const int64_t v = uni(-6, 20);
        if (wide) c.v64.push_back(v); else c.v32.push_back((int32_t)v);
        const int64_t s = i ? c.ends[i - 1] : 0;
        for (int64_t k = s; k < c.ends[i]; ++k) c.rows.push_back(v);
    }
    c.d.enc = 1;
    c.d.vtype = wide ? 2 : 1;
    c.d.n = (int64_t)c.ends.size();
    c.d.values = wide ? (const void*)c.v64.data() : (const void*)c.v32.data();
    c.d.run_ends = c.ends.data();
    return c;
}

Col make_index(int64_t n, bool wide_pos) {
    Col c;
    c.rows.assign(n, 0);
    for (int64_t r = 0; r < n; ++r)
        if (rng() % 4 == 0) {
            const int64_t v = uni(-50, 50);
            if (wide_pos) c.p64.push_back(r); else c.p32.push_back((int32_t)r);
            c.v64.push_back(v);
            c.rows[r] = v;
        }
    c.d.enc = 2;
    c.d.vtype = 2;
    c.d.ptype = wide_pos ? 2 : 1;
    c.d.n = (int64_t)c.v64.size();
    c.d.values = c.v64.data();
    c.d.positions = wide_pos ? (const void*)c.p64.data() : (const void*)c.p32.data();
    return c;
}

Col make_packed(int64_t n, int w, int64_t base) {
    Col c;
    c.packed.assign((size_t)((n * w + 31) / 32 + 2), 0u);
    for (int64_t r = 0; r < n; ++r) {
        const uint64_t code = w == 32 ? (uint64_t)(uint32_t)rng() : (rng() & ((1ull << w) - 1));
        const uint64_t bit = (uint64_t)r * w;
        for (int b = 0; b < w; ++b)
            if ((code >> b) & 1) c.packed[(bit + b) >> 5] |= 1u << ((bit + b) & 31);
        c.rows.push_back(base + (int64_t)code);
    }
    c.d.enc = 3;
    c.d.n = n;
    c.d.packed = c.packed.data();
    c.d.w = w;
    c.d.base = base;
    return c;
}

// RLE + Index: pure runs of 2-8 rows and single rows listed as points
Col make_rle_index(int64_t n, bool wide_pos) {
    Col c;
    c.rows.assign(n, 0);
    int64_t r = 0;
    while (r < n) {
        const int64_t v = uni(-6, 20);
        if (rng() % 3 == 0 || r + 2 > n) {
            if (wide_pos) c.p64.push_back(r); else c.p32.push_back((int32_t)r);
            c.pv.push_back(v);
            c.rows[r++] = v;
        } else {
            const int64_t e = std::min(n, r + uni(2, 9));
            c.v64.push_back(v);
            c.starts.push_back(r);
            c.ends.push_back(e);
            for (; r < e; ++r) c.rows[r] = v;
        }
    }
    c.d.enc = 4;
    c.d.vtype = 2;
    c.d.n = (int64_t)c.ends.size();
    c.d.values = c.v64.data();
    c.d.run_starts = c.starts.data();
    c.d.run_ends = c.ends.data();
    c.d.pt_n = (int64_t)c.pv.size();
    c.d.pt_ptype = wide_pos ? 2 : 1;
    c.d.pt_vtype = 2;
    c.d.pt_positions = wide_pos ? (const void*)c.p64.data() : (const void*)c.p32.data();
    c.d.pt_values = c.pv.data();
    return c;
}

// Plain + Index: 6-bit codes, about one row in five an outlier point
Col make_plain_index(int64_t n) {
    Col c = make_packed(n, 6, -10);
    for (int64_t r = 0; r < n; ++r)
        if (rng() % 5 == 0) {
            const int64_t v = uni(-1000, 1000);
            c.p32.push_back((int32_t)r);
            c.pv.push_back(v);
            c.rows[r] = v;
        }
    c.d.enc = 5;
    c.d.pt_n = (int64_t)c.pv.size();
    c.d.pt_ptype = 1;
    c.d.pt_vtype = 2;
    c.d.pt_positions = c.p32.data();
    c.d.pt_values = c.pv.data();
    return c;
}

}  // namespace

int main() {
    int checked = 0;
    for (int t = 0; t < 60; ++t) {
        const int64_t n = uni(1, 3000);
        std::vector<Col> cols;
        cols.push_back(make_rle(n, t % 2));
        cols.push_back(make_rle(n, false));
        cols.push_back(make_index(n, t % 3 == 0));
        const int w = 1 + t % 32;
        cols.push_back(make_packed(n, w, t % 2 ? -(int64_t(1) << (w - 1)) : 0));
        cols.push_back(make_rle_index(n, t % 2 == 0));
        cols.push_back(make_plain_index(n));
        std::vector<orc_column> d;
        for (auto& c : cols) d.push_back(c.d);
        for (int qi = 0; qi < 6; ++qi) {
            std::vector<std::vector<int64_t>> lists;
            std::vector<orc_pred> preds;
            const int np = (int)uni(0, 4);
            for (int i = 0; i < np; ++i) {
                orc_pred p{};
                p.col = (int)uni(0, 6);
                p.op = (int)uni(1, 5);
                p.lo = uni(-10, 15);
                p.hi = p.lo + uni(0, 20);
                lists.push_back({uni(-5, 20), uni(-5, 20), uni(-5, 20)});
                p.clause = (int)uni(0, 3);
                preds.push_back(p);
            }
            for (size_t i = 0; i < preds.size(); ++i) {
                preds[i].in_list = lists[i].data();
                preds[i].in_len = (int64_t)lists[i].size();
            }
            std::vector<orc_key> keys;
            if (rng() % 2) keys.push_back({1, 0, 32});       // values of column 1 lie in [-6, 20): some out of
                                                           // the domain, which the oracle reports as an error
            std::vector<orc_agg> aggs = {{1, -1, 0, 0}, {2, 2, 0, 0}, {3, 0, 0, 0}, {4, 3, 0, 0},
                                         {2, 0, 1, 1}, {3, 3, 3, 1}, {4, 0, 2, 2}, {2, 4, 1, 5}};
            if (rng() % 2) aggs.back() = {3, 5, 0, 0};
            const int64_t rb = uni(0, n), re = uni(rb, n + 1);
            const int threads = 1 + (int)uni(0, 4);
            void* h = orc_query(d.data(), (int32_t)d.size(), n, preds.data(), (int32_t)preds.size(), keys.data(),
                                (int32_t)keys.size(), aggs.data(), (int32_t)aggs.size(), rb, re, threads);
            // the driver's own evaluation, row by row
            auto holds = [&](const orc_pred& p, int64_t r) {
                const int64_t v = cols[p.col].rows[r];
                bool h_;
                if (p.op == 1 || p.op == 3) h_ = p.lo <= v && v < p.hi;
                else {
                    h_ = false;
                    for (int64_t k = 0; k < p.in_len; ++k) h_ = h_ || p.in_list[k] == v;
                }
                return (p.op == 3 || p.op == 4) ? !h_ : h_;
            };
            std::map<std::vector<int64_t>, std::vector<int64_t>> groups;
            bool domain_error = false;
            for (int64_t r = rb; r < re; ++r) {
                bool pass = true;
                std::map<int32_t, bool> any;
                for (auto& p : preds) {
                    if (p.clause == 0) pass = pass && holds(p, r);
                    else any[p.clause] = any[p.clause] || holds(p, r);
                }
                for (auto& kv : any) pass = pass && kv.second;
                if (!pass) continue;
                std::vector<int64_t> key;
                for (auto& k : keys) {
                    const int64_t v = cols[k.col].rows[r] >> k.shift;
                    if (v < 0 || v >= k.card) domain_error = true;
                    key.push_back(v);
                }
                auto& acc = groups[key];
                if (acc.empty()) {
                    acc.assign(1 + aggs.size(), 0);
                    for (size_t a = 0; a < aggs.size(); ++a)
                        acc[1 + a] = aggs[a].func == 3 ? INT64_MAX : aggs[a].func == 4 ? INT64_MIN : 0;
                }
                acc[0] += 1;
                for (size_t a = 0; a < aggs.size(); ++a) {
                    int64_t x = 1;
                    if (aggs[a].func != 1) {
                        x = cols[aggs[a].col].rows[r];
                        const int64_t y = cols[aggs[a].col2].rows[r];
                        if (aggs[a].op == 1) x += y;
                        if (aggs[a].op == 2) x -= y;
                        if (aggs[a].op == 3) x *= y;
                    }
                    int64_t& v = acc[1 + a];
                    v = aggs[a].func == 3 ? std::min(v, x) : aggs[a].func == 4 ? std::max(v, x) : v + x;
                }
            }
            const char* err = orc_error(h);
            if (domain_error) {
                if (!err || !*err) { fprintf(stderr, "expected a domain error\n"); return 1; }
            } else {
                if (err && *err) { fprintf(stderr, "oracle error: %s\n", err); return 1; }
                const int64_t g = orc_n_groups(h);
                std::vector<int64_t> kb(std::max<int64_t>(1, g * (int64_t)keys.size())), cb(std::max<int64_t>(1, g)),
                    ab(std::max<int64_t>(1, g * (int64_t)aggs.size()));
                orc_copy(h, kb.data(), cb.data(), ab.data());
                if (keys.empty()) {
                    const auto it = groups.find({});
                    const int64_t cnt = it == groups.end() ? 0 : it->second[0];
                    if (g != 1 || cb[0] != cnt) { fprintf(stderr, "ungrouped count differs\n"); return 1; }
                    for (size_t a = 0; a < aggs.size(); ++a)
                        if (ab[a] != (cnt ? it->second[1 + a] : 0)) { fprintf(stderr, "aggregate differs\n"); return 1; }
                } else {
                    if (g != (int64_t)groups.size()) { fprintf(stderr, "group count differs\n"); return 1; }
                    int64_t i = 0;
                    for (auto& kv : groups) {
                        if (kb[i] != kv.first[0] || cb[i] != kv.second[0]) { fprintf(stderr, "group differs\n"); return 1; }
                        for (size_t a = 0; a < aggs.size(); ++a)
                            if (ab[i * aggs.size() + a] != kv.second[1 + a]) { fprintf(stderr, "group aggregate differs\n"); return 1; }
                        ++i;
                    }
                }
            }
            orc_free(h);
            ++checked;
        }
    }
    printf("sanitized oracle: %d queries checked\n", checked);
    return 0;
}
