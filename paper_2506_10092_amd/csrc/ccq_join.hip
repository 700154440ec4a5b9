// Joins on encoded columns (Section 8): Get Join Index and Apply Join Index.
//
// A join entry is a run of an RLE column (value, row range clipped to the
// window), a listed point of an Index column, or one row of a bit-packed
// column.  Get Join Index hashes the right column's entries by value into an
// open-addressing table in device memory: a slot is claimed by a 64-bit
// compare-and-swap of its key (no spin waits; the one value that equals the
// empty marker has a slot of its own), and the entries of one value form a
// chain through an atomic exchange of the slot's head, with the chain's
// entry count and row count kept per slot.  Each left entry then finds its
// value's slot: the count pass gives its number of blocks (the chain's
// entries) and pairs (its length times the chain's rows), a scan gives the
// offsets, and the write pass walks the chain writing one block per match,
// the cross product of the two entries' row ranges (an RLE side keeps row
// ranges, Table 6).  The order of blocks within one left entry follows the
// chain (the paper's Join Index tensors are unsorted).
//
// Apply Join Index reads one side's column at the rows of every pair, block
// by block (left row outer): a scan of the blocks' pair counts, then one
// thread per output value finding its block by binary search and decoding
// the column at that row.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "ccq_internal.h"

namespace ccq {
namespace {

constexpr int kJThreads = 256;
constexpr int64_t kMaxGrid = 8192;        // workgroups of the grid-stride kernels
constexpr int64_t kEmpty = INT64_MIN;     // empty slot marker (the value INT64_MIN uses slot cap)

struct JCol {                  // one side's column and window
    int32_t enc;               // CCQ_RLE, CCQ_INDEX, CCQ_BITPACKED
    int32_t vtype, ptype;
    int32_t w;
    int64_t base;
    const void* vals;
    const int64_t* ends;
    const void* pos;
    const uint32_t* packed;
    int64_t n;                 // runs / points / rows of the column
    int64_t begin, end;        // window
    int64_t first;             // first entry inside the window (device-computed)
};

__device__ __forceinline__ int64_t jld(const void* p, int32_t t, int64_t i) {
    return t == CCQ_I32 ? (int64_t)((const int32_t*)p)[i] : ((const int64_t*)p)[i];
}

__device__ __forceinline__ int64_t packed_value(const JCol& c, int64_t r) {
    const uint64_t bit = (uint64_t)r * (uint64_t)c.w;
    const uint64_t two = (uint64_t)c.packed[bit >> 5] | ((uint64_t)c.packed[(bit >> 5) + 1] << 32);
    const uint64_t mask = c.w == 32 ? 0xFFFFFFFFull : ((1ull << c.w) - 1ull);
    return c.base + (int64_t)((two >> (bit & 31)) & mask);
}

// entry k (k from c.first): value, first row, rows
__device__ __forceinline__ void entry(const JCol& c, int64_t k, int64_t* v, int64_t* s, int64_t* len) {
    if (c.enc == CCQ_RLE) {
        const int64_t i = c.first + k;
        const int64_t rs = i > 0 ? c.ends[i - 1] : 0;
        const int64_t a = max(rs, c.begin), b = min(c.ends[i], c.end);
        *v = jld(c.vals, c.vtype, i);
        *s = a;
        *len = b - a;
    } else if (c.enc == CCQ_INDEX) {
        const int64_t i = c.first + k;
        *v = jld(c.vals, c.vtype, i);
        *s = jld(c.pos, c.ptype, i);
        *len = 1;
    } else {
        const int64_t r = c.begin + k;
        *v = packed_value(c, r);
        *s = r;
        *len = 1;
    }
}

__device__ __forceinline__ uint64_t mix(int64_t v) {
    uint64_t x = (uint64_t)v;
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// Window bounds of both sides: first entry and entry count (one thread).
__device__ int64_t upper_bound_dev(const int64_t* a, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (a[m] > x) hi = m; else lo = m + 1;
    }
    return lo;
}

__device__ int64_t lower_bound_pos(const void* p, int32_t t, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (jld(p, t, m) < x) lo = m + 1; else hi = m;
    }
    return lo;
}

__device__ void bounds(const JCol& c, int64_t* first, int64_t* count) {
    if (c.end <= c.begin) {
        *first = 0;
        *count = 0;
    } else if (c.enc == CCQ_RLE) {
        *first = upper_bound_dev(c.ends, c.n, c.begin);
        *count = upper_bound_dev(c.ends, c.n, c.end - 1) + 1 - *first;
    } else if (c.enc == CCQ_INDEX) {
        *first = lower_bound_pos(c.pos, c.ptype, c.n, c.begin);
        *count = lower_bound_pos(c.pos, c.ptype, c.n, c.end) - *first;
    } else {
        *first = 0;
        *count = c.end - c.begin;
    }
}

__global__ void k_join_bounds(JCol l, JCol r, int64_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        bounds(l, &out[0], &out[1]);
        bounds(r, &out[2], &out[3]);
    }
}

struct JTable {
    int64_t* keys;             // [cap + 1]; slot cap holds the value kEmpty
    int64_t* head;             // [cap + 1] first right entry of the slot's chain, -1 if none
    unsigned long long* cnt;   // [cap + 1] right entries of the slot
    unsigned long long* rows;  // [cap + 1] their rows
    int64_t* next;             // [n_right] chain links
    int64_t cap;               // power of two
};

__global__ void k_join_clear(JTable T) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= T.cap; i += stride) {
        T.keys[i] = kEmpty;
        T.head[i] = -1;
        T.cnt[i] = 0;
        T.rows[i] = 0;
    }
}

// the slot of value v: claim an empty one or find v's (insert = true), or
// find v's only (-1 if absent)
__device__ __forceinline__ int64_t slot_of(const JTable& T, int64_t v, bool insert) {
    if (v == kEmpty) return T.cap;
    const int64_t mask = T.cap - 1;
    int64_t s = (int64_t)(mix(v) & (uint64_t)mask);
    for (int64_t probes = 0; probes <= mask; ++probes, s = (s + 1) & mask) {
        if (insert) {
            const unsigned long long old =
                atomicCAS((unsigned long long*)&T.keys[s], (unsigned long long)kEmpty, (unsigned long long)v);
            if ((int64_t)old == kEmpty || (int64_t)old == v) return s;
        } else {
            const int64_t k = T.keys[s];
            if (k == v) return s;
            if (k == kEmpty) return -1;
        }
    }
    return -1;      // table full (cannot happen: cap >= 2 * entries)
}

__global__ void k_join_build(JTable T, JCol r, int64_t n_right) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_right; k += stride) {
        int64_t v, s, len;
        entry(r, k, &v, &s, &len);
        const int64_t slot = slot_of(T, v, true);
        if (slot < 0) continue;
        T.next[k] = (int64_t)atomicExch((unsigned long long*)&T.head[slot], (unsigned long long)k);
        atomicAdd(&T.cnt[slot], 1ull);
        atomicAdd(&T.rows[slot], (unsigned long long)len);
    }
}

// per left entry: its blocks (counts[k]); per workgroup: its entries' pairs (ppart[block])
__global__ __launch_bounds__(kJThreads) void k_join_count(JTable T, JCol l, int64_t n_left, int64_t* counts,
                                                          unsigned long long* ppart) {
    __shared__ unsigned long long sw[kJThreads / 64];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long p = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_left; k += stride) {
        int64_t v, s, len;
        entry(l, k, &v, &s, &len);
        const int64_t slot = slot_of(T, v, false);
        counts[k] = slot < 0 ? 0 : (int64_t)T.cnt[slot];
        if (slot >= 0) p += (unsigned long long)len * T.rows[slot];
    }
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kJThreads / 64; ++w) t += sw[w];
        ppart[blockIdx.x] = t;
    }
}

// the sum of n partials into *total (one workgroup)
__global__ __launch_bounds__(kJThreads) void k_sum_parts(const unsigned long long* part, int64_t n,
                                                         unsigned long long* total) {
    __shared__ unsigned long long sw[kJThreads / 64];
    unsigned long long p = 0;
    for (int64_t i = threadIdx.x; i < n; i += kJThreads) p += part[i];
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kJThreads / 64; ++w) t += sw[w];
        *total = t;
    }
}

__global__ void k_join_write(JTable T, JCol l, JCol r, int64_t n_left, const int64_t* offsets,
                             ccq_join_block* out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_left; k += stride) {
        int64_t v, s, len;
        entry(l, k, &v, &s, &len);
        const int64_t slot = slot_of(T, v, false);
        if (slot < 0) continue;
        int64_t o = offsets[k];
        for (int64_t j = T.head[slot]; j >= 0; j = T.next[j]) {
            int64_t rv, rs, rl;
            entry(r, j, &rv, &rs, &rl);
            ccq_join_block b;
            b.left_start = s;
            b.left_len = len;
            b.right_start = rs;
            b.right_len = rl;
            out[o++] = b;
        }
    }
}

// ---- exclusive scan of an int64 array (three launches)

constexpr int64_t kScanPer = 4096;

__device__ __forceinline__ int64_t blk_incl(int64_t x, int64_t* sw, int64_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) sw[wave] = x;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < kJThreads / 64; ++w) {
        if (w < wave) before += sw[w];
        all += sw[w];
    }
    __syncthreads();
    *total = all;
    return x + before;
}

// per chunk of kScanPer entries: its total
__global__ void k_scan_part(const int64_t* in, int64_t n, int64_t* part) {
    __shared__ int64_t sw[kJThreads / 64];
    const int64_t c0 = (int64_t)blockIdx.x * kScanPer;
    int64_t x = 0;
    for (int64_t i = c0 + threadIdx.x; i < min(n, c0 + kScanPer); i += kJThreads) x += in[i];
    int64_t t;
    blk_incl(x, sw, &t);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// exclusive scan of the chunk totals in place, the grand total at part[nb]
__global__ void k_scan_parts(int64_t* part, int64_t nb) {
    __shared__ int64_t sw[kJThreads / 64];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kJThreads) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t x = b < nb ? part[b] : 0;
        int64_t all;
        const int64_t inc = blk_incl(x, sw, &all);
        if (b < nb) part[b] = carry + inc - x;
        carry += all;
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

// out[i] = exclusive prefix of in at i (chunk offset + in-chunk scan)
__global__ void k_scan_final(const int64_t* in, int64_t n, const int64_t* part, int64_t* out) {
    __shared__ int64_t sw[kJThreads / 64];
    const int64_t c0 = (int64_t)blockIdx.x * kScanPer;
    int64_t carry = part[blockIdx.x];
    for (int64_t b0 = c0; b0 < min(n, c0 + kScanPer); b0 += kJThreads) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t x = i < n ? in[i] : 0;
        int64_t all;
        const int64_t inc = blk_incl(x, sw, &all);
        if (i < n) out[i] = carry + inc - x;
        carry += all;
    }
}

// ---- Apply Join Index

// pair counts of the blocks; a block whose rows on `side` leave [0, n_rows)
// or whose lengths are negative counts 0 and raises *bad
__global__ void k_pair_counts(const ccq_join_block* b, int64_t n, int32_t side, int64_t n_rows, int64_t* pc,
                              int32_t* bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const ccq_join_block x = b[i];
        const int64_t s0 = side == 0 ? x.left_start : x.right_start;
        const int64_t l0 = side == 0 ? x.left_len : x.right_len;
        const bool okb = x.left_len >= 0 && x.right_len >= 0 && s0 >= 0 && s0 <= n_rows && l0 <= n_rows - s0;
        if (!okb) *bad = 1;
        pc[i] = okb ? x.left_len * x.right_len : 0;
    }
}

// the value of column c at row r (an Index column holds 0 at rows it does not list)
__device__ __forceinline__ int64_t value_at_row(const JCol& c, int64_t r) {
    if (c.enc == CCQ_RLE) return jld(c.vals, c.vtype, upper_bound_dev(c.ends, c.n, r));
    if (c.enc == CCQ_INDEX) {
        const int64_t i = lower_bound_pos(c.pos, c.ptype, c.n, r);
        return (i < c.n && jld(c.pos, c.ptype, i) == r) ? jld(c.vals, c.vtype, i) : 0;
    }
    return packed_value(c, r);
}

constexpr int kApplyPer = 16;                               // consecutive outputs per thread
constexpr int64_t kApplyChunk = (int64_t)kJThreads * kApplyPer;  // outputs per workgroup

// last block m in [lo, hi] with off[m] <= p (off[lo] <= p)
__device__ __forceinline__ int64_t block_of(const int64_t* off, int64_t lo, int64_t hi, int64_t p) {
    while (lo < hi) {
        const int64_t m = (lo + hi + 1) >> 1;
        if (off[m] <= p) lo = m; else hi = m - 1;
    }
    return lo;
}

// reads a column at rows that mostly step by one: an RLE cursor keeps the
// current run, an Index cursor the next listed point
struct RowCursor {
    int64_t i = -1, lo = 0, hi = 0;    // RLE: run i covers [lo, hi); Index: point i is the first >= hi - 1
    int64_t v = 0;
};

__device__ __forceinline__ int64_t read_row(const JCol& c, int64_t r, RowCursor& k) {
    if (c.enc == CCQ_RLE) {
        if (k.i < 0 || r < k.lo || r >= k.hi) {
            if (k.i >= 0 && r == k.hi) ++k.i; else k.i = upper_bound_dev(c.ends, c.n, r);
            k.lo = k.i > 0 ? c.ends[k.i - 1] : 0;
            k.hi = c.ends[k.i];
            k.v = jld(c.vals, c.vtype, k.i);
        }
        return k.v;
    }
    if (c.enc == CCQ_INDEX) {
        // k.lo: the row last read; k.i: the first point at or after it
        if (k.i < 0 || r != k.lo + 1) k.i = lower_bound_pos(c.pos, c.ptype, c.n, r);
        else if (k.i < c.n && jld(c.pos, c.ptype, k.i) < r) ++k.i;
        k.lo = r;
        return (k.i < c.n && jld(c.pos, c.ptype, k.i) == r) ? jld(c.vals, c.vtype, k.i) : 0;
    }
    return packed_value(c, r);
}

// the block holding each chunk's first output (one thread per chunk, all
// searches in flight together); entry n_chunks holds the last output's block
__global__ void k_chunk_first(const int64_t* off, int64_t nb, int64_t total, int64_t n_chunks, int64_t* first) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n_chunks; c += stride)
        first[c] = block_of(off, 0, nb - 1, min(c * kApplyChunk, total - 1));
}

constexpr int kApplyLds = 2048;            // block offsets a workgroup stages in LDS

// one workgroup per chunk of kApplyChunk outputs; each thread takes
// kApplyPer consecutive ones (one block search and one division, the rows,
// then all their loads), stages them in LDS, and the chunk is written with
// coalesced stores
__global__ __launch_bounds__(kJThreads) void k_join_apply(const ccq_join_block* b, int64_t nb, const int64_t* off,
                                                          int64_t total, const int64_t* first, JCol c, int32_t side,
                                                          int64_t* out) {
    // padded by one slot per kApplyPer: a thread's run starts 17 slots after its neighbour's
    __shared__ int64_t sout[kApplyChunk + kApplyChunk / kApplyPer];
    __shared__ int64_t soff[kApplyLds];
    const int64_t c0 = (int64_t)blockIdx.x * kApplyChunk;
    const int64_t c1 = min(total, c0 + kApplyChunk);
    // the chunk's blocks lie in [lo, hi]
    const int64_t lo = first[blockIdx.x], hi = first[blockIdx.x + 1];
    const bool staged = hi - lo < kApplyLds;
    if (staged)
        for (int64_t i = threadIdx.x; i <= hi - lo; i += kJThreads) soff[i] = off[lo + i];
    __syncthreads();
    const int64_t p0 = c0 + (int64_t)threadIdx.x * kApplyPer;
    if (p0 < c1) {
        int64_t k;
        if (staged) {
            int32_t a = 0, z = (int32_t)(hi - lo);
            while (a < z) {
                const int32_t m = (a + z + 1) >> 1;
                if (soff[m] <= p0) a = m; else z = m - 1;
            }
            k = lo + a;
        } else {
            k = block_of(off, lo, hi, p0);
        }
        // k holds pair p0: blocks of no pairs share the next one's offset and are never last
        ccq_join_block bb = b[k];
        const int64_t q = p0 - off[k];
        int64_t a = q / bb.right_len, r = q % bb.right_len;
        const int n = (int)min<int64_t>(kApplyPer, c1 - p0);
        int64_t rows[kApplyPer];
#pragma unroll
        for (int j = 0; j < kApplyPer; ++j) {
            rows[j] = side == 0 ? bb.left_start + a : bb.right_start + r;
            if (++r == bb.right_len) {
                r = 0;
                if (++a == bb.left_len && j + 1 < n) {
                    // next block with pairs (one exists: pair p0 + j + 1 < total)
                    do {
                        bb = b[++k];
                    } while (bb.left_len == 0 || bb.right_len == 0);
                    a = 0;
                }
            }
        }
        int64_t* dst = sout + threadIdx.x * (kApplyPer + 1);
        if (c.enc == CCQ_BITPACKED) {
            // independent loads, all in flight together
#pragma unroll
            for (int j = 0; j < kApplyPer; ++j)
                if (j < n) dst[j] = packed_value(c, rows[j]);
        } else {
            RowCursor cur;
#pragma unroll
            for (int j = 0; j < kApplyPer; ++j)
                if (j < n) dst[j] = read_row(c, rows[j], cur);
        }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < c1 - c0; i += kJThreads) out[c0 + i] = sout[i + i / kApplyPer];
}

// ---- host helpers

ccq_status jcol(const ccq_table* t, int32_t col, int64_t begin, int64_t end, JCol* c) {
    if (!t) return fail(CCQ_E_INVALID, "table is NULL");
    if (col < 0 || col >= (int32_t)t->cols.size()) return fail(CCQ_E_INVALID, "column %d out of range", col);
    if (begin < 0 || end > t->n_rows || begin > end) return fail(CCQ_E_INVALID, "window outside the table");
    const ccq_column_desc& d = t->cols[col];
    if (d.encoding != CCQ_RLE && d.encoding != CCQ_INDEX && d.encoding != CCQ_BITPACKED)
        return fail(CCQ_E_UNSUPPORTED, "column %d: joins take RLE, INDEX and BITPACKED columns", col);
    memset(c, 0, sizeof *c);
    c->enc = d.encoding;
    c->vtype = d.value_type;
    c->ptype = d.position_type;
    c->w = d.bit_width;
    c->base = d.base;
    c->vals = d.values;
    c->ends = d.run_ends;
    c->pos = d.positions;
    c->packed = d.packed;
    c->n = d.encoding == CCQ_BITPACKED ? t->n_rows : d.n_entries;
    c->begin = begin;
    c->end = end;
    return CCQ_OK;
}

int64_t max_entries(const JCol& c) { return c.enc == CCQ_BITPACKED ? c.end - c.begin : c.n; }

int64_t table_cap(int64_t n_right) {
    int64_t cap = 64;
    while (cap < 2 * n_right) cap <<= 1;
    return cap;
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct JWs {
    JTable T;
    int64_t* bounds;         // [4]
    unsigned long long* pairs;
    int64_t* counts;         // [n_left]
    int64_t* offsets;        // [n_left]
    int64_t* part;           // [chunks + 1]
    unsigned long long* ppart;  // [count grid] pairs per workgroup
    size_t total;
};

JWs join_ws(unsigned char* base, int64_t n_left, int64_t n_right) {
    JWs w;
    const int64_t cap = table_cap(n_right);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base ? base + o : nullptr;
        o += a256(bytes);
        return p;
    };
    w.bounds = (int64_t*)take(64);
    w.pairs = (unsigned long long*)take(8);
    w.T.cap = cap;
    w.T.keys = (int64_t*)take(8 * (size_t)(cap + 1));
    w.T.head = (int64_t*)take(8 * (size_t)(cap + 1));
    w.T.cnt = (unsigned long long*)take(8 * (size_t)(cap + 1));
    w.T.rows = (unsigned long long*)take(8 * (size_t)(cap + 1));
    w.T.next = (int64_t*)take(8 * (size_t)std::max<int64_t>(n_right, 1));
    w.counts = (int64_t*)take(8 * (size_t)std::max<int64_t>(n_left, 1));
    w.offsets = (int64_t*)take(8 * (size_t)std::max<int64_t>(n_left, 1));
    w.part = (int64_t*)take(8 * (size_t)((n_left + kScanPer - 1) / kScanPer + 2));
    w.ppart = (unsigned long long*)take(8 * (size_t)kMaxGrid);
    w.total = o;
    return w;
}

unsigned grid_for(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kJThreads - 1) / kJThreads, kMaxGrid));
}

// exclusive scan of in[n] into out[n]; the total lands at part[chunks]
void scan(const int64_t* in, int64_t n, int64_t* part, int64_t* out, hipStream_t s) {
    const int64_t chunks = std::max<int64_t>(1, (n + kScanPer - 1) / kScanPer);
    hipLaunchKernelGGL(k_scan_part, dim3((unsigned)chunks), dim3(kJThreads), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kJThreads), 0, s, part, chunks);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)chunks), dim3(kJThreads), 0, s, in, n, part, out);
}

}  // namespace
}  // namespace ccq

using namespace ccq;

extern "C" {

size_t ccq_join_workspace_bytes(const ccq_table* left, int32_t left_col, int64_t left_begin, int64_t left_end,
                                const ccq_table* right, int32_t right_col, int64_t right_begin, int64_t right_end) {
    JCol l, r;
    if (jcol(left, left_col, left_begin, left_end, &l) || jcol(right, right_col, right_begin, right_end, &r))
        return 0;
    return join_ws(nullptr, max_entries(l), max_entries(r)).total;
}

ccq_status ccq_join_index(const ccq_table* left, int32_t left_col, int64_t left_begin, int64_t left_end,
                          const ccq_table* right, int32_t right_col, int64_t right_begin, int64_t right_end, void* ws,
                          size_t ws_bytes, void* stream, ccq_join_block* blocks, int64_t capacity, int64_t* n_blocks,
                          int64_t* n_pairs) {
    if (!n_blocks || !n_pairs) return fail(CCQ_E_INVALID, "n_blocks / n_pairs is NULL");
    *n_blocks = *n_pairs = 0;
    JCol l, r;
    if (ccq_status st = jcol(left, left_col, left_begin, left_end, &l)) return st;
    if (ccq_status st = jcol(right, right_col, right_begin, right_end, &r)) return st;
    if (left->ctx->device < 0 || left->ctx->device != right->ctx->device)
        return fail(CCQ_E_INVALID, "both tables need a device context on one device");
    if (!ws || ((uintptr_t)ws & 255)) return fail(CCQ_E_INVALID, "workspace must be 256-byte aligned");
    const JWs w = join_ws((unsigned char*)ws, max_entries(l), max_entries(r));
    if (ws_bytes < w.total) return fail(CCQ_E_CAPACITY, "workspace of %zu bytes, %zu needed", ws_bytes, w.total);
    hipError_t e = hipSetDevice(left->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    // entries inside the windows
    hipLaunchKernelGGL(k_join_bounds, dim3(1), dim3(64), 0, s, l, r, w.bounds);
    int64_t b[4];
    e = hipMemcpyAsync(b, w.bounds, sizeof b, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "join bounds");
    l.first = b[0];
    r.first = b[2];
    const int64_t nl = b[1], nr = b[3];
    // build on the right entries, count the left ones' matches
    hipLaunchKernelGGL(k_join_clear, dim3(grid_for(w.T.cap + 1)), dim3(kJThreads), 0, s, w.T);
    e = hipMemsetAsync(w.pairs, 0, 8, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    if (nr > 0) hipLaunchKernelGGL(k_join_build, dim3(grid_for(nr)), dim3(kJThreads), 0, s, w.T, r, nr);
    if (nl > 0) {
        const unsigned g = grid_for(nl);
        hipLaunchKernelGGL(k_join_count, dim3(g), dim3(kJThreads), 0, s, w.T, l, nl, w.counts, w.ppart);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kJThreads), 0, s, w.ppart, (int64_t)g, w.pairs);
        scan(w.counts, nl, w.part, w.offsets, s);
    }
    int64_t tot = 0;
    unsigned long long pairs = 0;
    const int64_t chunks = std::max<int64_t>(1, (nl + kScanPer - 1) / kScanPer);
    if (nl > 0) e = hipMemcpyAsync(&tot, w.part + chunks, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&pairs, w.pairs, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "join count");
    *n_blocks = tot;
    *n_pairs = (int64_t)pairs;
    if (tot > capacity) return fail(CCQ_E_CAPACITY, "%lld blocks, capacity %lld", (long long)tot, (long long)capacity);
    if (tot > 0) {
        if (!blocks) return fail(CCQ_E_INVALID, "blocks is NULL");
        hipLaunchKernelGGL(k_join_write, dim3(grid_for(nl)), dim3(kJThreads), 0, s, w.T, l, r, nl, w.offsets, blocks);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "join write");
    return ok();
}

size_t ccq_join_apply_workspace_bytes(int64_t n_blocks, int64_t n_pairs) {
    const int64_t n = std::max<int64_t>(n_blocks, 1);
    const int64_t chunks = std::max<int64_t>(n_pairs, 0) / kApplyChunk + 2;
    return 256 + a256(8 * (size_t)n) * 2 + a256(8 * (size_t)((n + kScanPer - 1) / kScanPer + 2)) +
           a256(8 * (size_t)chunks);
}

ccq_status ccq_join_apply(const ccq_table* t, int32_t col, const ccq_join_block* blocks, int64_t n_blocks, int32_t side,
                          void* ws, size_t ws_bytes, void* stream, int64_t* out, int64_t capacity, int64_t* n_out) {
    if (!n_out) return fail(CCQ_E_INVALID, "n_out is NULL");
    *n_out = 0;
    JCol c;
    if (ccq_status st = jcol(t, col, 0, t ? t->n_rows : 0, &c)) return st;
    if (t->ctx->device < 0) return fail(CCQ_E_INVALID, "a device context is required");
    if (side != 0 && side != 1) return fail(CCQ_E_INVALID, "side must be 0 (left) or 1 (right)");
    if (n_blocks < 0 || (n_blocks > 0 && !blocks)) return fail(CCQ_E_INVALID, "bad block list");
    if (!ws || ((uintptr_t)ws & 255)) return fail(CCQ_E_INVALID, "workspace must be 256-byte aligned");
    if (ws_bytes < ccq_join_apply_workspace_bytes(n_blocks, 0)) return fail(CCQ_E_CAPACITY, "workspace too small");
    if (n_blocks == 0) return ok();
    hipError_t e = hipSetDevice(t->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = n_blocks;
    unsigned char* w = (unsigned char*)ws;
    int32_t* bad = (int32_t*)w;
    int64_t* pc = (int64_t*)(w + 256);
    int64_t* off = (int64_t*)(w + 256 + a256(8 * (size_t)n));
    int64_t* part = (int64_t*)(w + 256 + 2 * a256(8 * (size_t)n));
    int64_t* cfirst = (int64_t*)(w + 256 + 2 * a256(8 * (size_t)n) + a256(8 * (size_t)((n + kScanPer - 1) / kScanPer + 2)));
    e = hipMemsetAsync(bad, 0, 4, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    hipLaunchKernelGGL(k_pair_counts, dim3(grid_for(n)), dim3(kJThreads), 0, s, blocks, n, side, t->n_rows, pc, bad);
    scan(pc, n, part, off, s);
    int64_t total = 0;
    int32_t flag = 0;
    const int64_t chunks = std::max<int64_t>(1, (n + kScanPer - 1) / kScanPer);
    e = hipMemcpyAsync(&total, part + chunks, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, bad, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "join apply count");
    if (flag) return fail(CCQ_E_INVALID, "a block's rows lie outside the table");
    *n_out = total;
    if (total > capacity) return fail(CCQ_E_CAPACITY, "%lld values, capacity %lld", (long long)total, (long long)capacity);
    if (ws_bytes < ccq_join_apply_workspace_bytes(n_blocks, total))
        return fail(CCQ_E_CAPACITY, "workspace of %zu bytes, %zu needed for %lld pairs", ws_bytes,
                    ccq_join_apply_workspace_bytes(n_blocks, total), (long long)total);
    if (total > 0) {
        if (!out) return fail(CCQ_E_INVALID, "out is NULL");
        const int64_t chunks_out = (total + kApplyChunk - 1) / kApplyChunk;
        if (chunks_out > INT32_MAX) return fail(CCQ_E_UNSUPPORTED, "more than 2^31 chunks of output");
        hipLaunchKernelGGL(k_chunk_first, dim3(grid_for(chunks_out + 1)), dim3(kJThreads), 0, s, off, n, total,
                           chunks_out, cfirst);
        hipLaunchKernelGGL(k_join_apply, dim3((unsigned)chunks_out), dim3(kJThreads), 0, s, blocks, n, off, total,
                           cfirst, c, side, out);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "join apply");
    return ok();
}

}  // extern "C"
