// Device code of the fused filter / align / aggregate path: helpers, the
// per-wavefront tile pipelines and the persistent kernels k_fused / k_batch
// (templates; instantiated per RLE-column bound in ccq_inst.hip).  Internal
// to libccq.
//
// One query runs as a short launch sequence on one stream:
//   k_prepare   clear the group table and the status word;
//   k_fused     the hot path, persistent; each wavefront is an independent
//               worker over a contiguous slice of the window;
//   finalize    the non-empty groups in key order into the result
//               (k_fin_single for ungrouped queries, else count/scan/write).
//
// Every path works on 2048-row tiles starting at multiples of 32 rows; lane
// l of a wave owns rows [32l, 32l + 32) of the tile, one 32-bit word of
// every row bitmap.  Three paths share that layout:
//   fast row path   one bit-packed column of width 14 or 20 (no RLE value
//                   per row): run batches are read straight from HBM, their
//                   predicate outcomes (a1) become toggle bitmaps whose
//                   prefix XOR is each column's pass mask (a2, a3); active
//                   lane-words are gathered into full batches and counted
//                   through an LDS code table into lane-replicated LDS
//                   counts (a4, a6, a7); Index points probe the pass bits
//                   (a5).  A software pipeline keeps the next tile's words
//                   and run batches in flight.
//   staged paths    the tile's runs are staged in LDS (stage_tile) with a
//                   run-boundary bitmap per column; the staged run holding
//                   row r is a prefix count plus a popcount (no search), the
//                   union of the columns' bitmaps is the aligned boundary
//                   set (a2), and toggles give the pass masks (a1, a3).
//     run mode      no bit-packed column: a lane cuts its word at the key
//                   and SUM columns' boundaries; each piece is an aligned
//                   run adding COUNT += rows and SUM += value * rows (a7).
//     generic rows  each lane walks its 32 rows; packed codes come from LDS-
//                   staged words (a4), RLE values from the advancing staged
//                   run, and rows of one group add up in registers before
//                   reaching a compact LDS group table (a6, a7).
#pragma once

#include "ccq_plan.h"

namespace ccq {

// ------------------------------------------------------------------ helpers

// Column data always lives in device global memory: reading it through the
// global address space gives global_load (counted by vmcnt only) instead of
// flat_load, whose completion every LDS wait would also have to await.
template <typename T>
__device__ __forceinline__ T gld(const T* p, int64_t i) {
    return ((const __attribute__((address_space(1))) T*)p)[i];
}

__device__ __forceinline__ int64_t ld_val(const void* p, int32_t vtype, int64_t i) {
    return vtype == 1 ? (int64_t)gld((const int32_t*)p, i) : gld((const int64_t*)p, i);
}

// The same without a branch on the type: always two dword loads (the high
// word of an int32 value reads its low word again), so that every path
// issues the same loads.
__device__ __forceinline__ int64_t ld_val_nb(const void* p, int32_t vtype, int64_t i) {
    const int32_t* q = (const int32_t*)p;
    const bool wide = vtype != 1;
    const int64_t k = wide ? 2 * i : i;
    const uint32_t lo = (uint32_t)gld(q, k);
    const uint32_t hi = (uint32_t)gld(q, wide ? k + 1 : k);
    return wide ? (int64_t)(((uint64_t)hi << 32) | lo) : (int64_t)(int32_t)lo;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// The wavefront's index in its workgroup, known to the compiler as
// wave-uniform (so everything derived from it stays in scalar registers).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

// number of set bits of m in the lanes below this one
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ __forceinline__ int wave_exclusive_sum(int v, int* total) {
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane_id() >= d) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - v;
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (no LDS): sums over 4, 8 and 16 lanes within each row of 16,
// then row 0's total into row 1, row 2's into row 3, and lane 31's into rows
// 2 and 3.
__device__ __forceinline__ int wave_inclusive_sum_dpp(int v) {
    int s = v + __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    s += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);          // row_shr:2
    s += __builtin_amdgcn_update_dpp(0, v, 0x113, 0xf, 0xf, true);          // row_shr:3
    s += __builtin_amdgcn_update_dpp(0, s, 0x114, 0xf, 0xe, false);         // row_shr:4, banks 1-3
    s += __builtin_amdgcn_update_dpp(0, s, 0x118, 0xf, 0xc, false);         // row_shr:8, banks 2-3
    s += __builtin_amdgcn_update_dpp(0, s, 0x142, 0xa, 0xf, false);         // row_bcast:15 into rows 1, 3
    s += __builtin_amdgcn_update_dpp(0, s, 0x143, 0xc, 0xf, false);         // row_bcast:31 into rows 2, 3
    return s;
}

// Cross-lane LDS hand-off inside one wavefront: a wave's LDS operations
// execute in order, so only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ bool set_contains(const int64_t* s, int32_t n, int64_t v) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (gld(s, mid) < v) lo = mid + 1; else hi = mid;
    }
    return lo < n && gld(s, lo) == v;
}

// v in one of n sorted, disjoint inclusive intervals (pairs lo, hi)
__device__ __forceinline__ bool intervals_contain(const int64_t* iv, int32_t n, int64_t v) {
    int32_t lo = 0, hi = n;   // first interval whose low end is > v
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (gld(iv, 2 * (int64_t)mid) <= v) lo = mid + 1; else hi = mid;
    }
    return lo > 0 && v <= gld(iv, 2 * (int64_t)(lo - 1) + 1);
}

__device__ __forceinline__ bool pred_pass(int32_t kind, int64_t lo, int64_t hi, const int64_t* set, int32_t n,
                                          int64_t v) {
    if (kind == kPredNone) return true;
    if (kind == kPredRange) return lo <= v && v < hi;
    if (kind == kPredNotRange) return v < lo || v >= hi;
    if (kind == kPredSet) return set_contains(set, n, v);
    if (kind == kPredIntervals) return intervals_contain(set, n, v);
    return false;
}

__device__ __forceinline__ void raise_status(int32_t* status, int32_t code) { atomicCAS(status, 0, code); }

// First index i in [0, n) with a[i] > x (n if none); the whole wave takes
// part and every lane gets the answer.  Each round probes 64 evenly spaced
// elements and keeps the stretch between the last probe <= x and the first
// probe > x.
__device__ inline int64_t wave_upper_bound(const int64_t* a, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    const int lane = lane_id();
    while (hi - lo > 64) {
        const int64_t len = hi - lo;
        const int64_t p = lo + ((int64_t)(lane + 1) * len) / 64 - 1;
        const uint64_t m = wave_ballot(gld(a, p) > x);
        if (m == 0) return hi;
        const int f = __builtin_ctzll(m);
        const int64_t nhi = lo + ((int64_t)(f + 1) * len) / 64 - 1;
        const int64_t nlo = f == 0 ? lo : lo + ((int64_t)f * len) / 64;
        lo = nlo;
        hi = nhi;
    }
    const int64_t i = lo + lane;
    const uint64_t m = wave_ballot(i < hi && gld(a, i) > x);
    return m ? lo + __builtin_ctzll(m) : hi;
}

// First index i in [0, n) with pos[i] >= x (n if none).
__device__ inline int64_t wave_lower_bound_pos(const void* pos, int32_t ptype, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    const int lane = lane_id();
    while (hi - lo > 64) {
        const int64_t len = hi - lo;
        const int64_t p = lo + ((int64_t)(lane + 1) * len) / 64 - 1;
        const uint64_t m = wave_ballot(ld_val(pos, ptype, p) >= x);
        if (m == 0) return hi;
        const int f = __builtin_ctzll(m);
        const int64_t nhi = lo + ((int64_t)(f + 1) * len) / 64 - 1;
        const int64_t nlo = f == 0 ? lo : lo + ((int64_t)f * len) / 64;
        lo = nlo;
        hi = nhi;
    }
    const int64_t i = lo + lane;
    const uint64_t m = wave_ballot(i < hi && ld_val(pos, ptype, i) >= x);
    return m ? lo + __builtin_ctzll(m) : hi;
}

// first index j in [0, n) with e[j] > x in an LDS array (n if none)
__device__ __forceinline__ int lds_upper_bound(const int32_t* e, int n, int32_t x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (e[mid] > x) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// ------------------------------------------------------------------ group table

// Dynamic LDS of the fused kernel.  Everything in it is addressed as this
// symbol plus an offset (never through a pointer that may be null), so the
// compiler keeps LDS accesses as ds_* instructions.
extern __shared__ __align__(16) unsigned char ccq_lds[];

struct Table {
    int64_t* g;                 // global: counts[G], then one [G] array per SUM
    int64_t G;
    int32_t loff;               // byte offset of the per-workgroup LDS copy, or -1
    int32_t c32;                // the LDS copy is compact: uint32 counts, int32 sums (below)
    int64_t lG;                 // groups [0, lG) have LDS cells
    uint64_t amap;              // compact table: LDS column of each accumulator (4 bits; 15: none)
};

// Add v to accumulator `which` (0: COUNT, 1 + k: SUM slot k) of group gid.
// A compact LDS table keeps 32-bit cells: counts cannot wrap (a workgroup
// counts fewer than 2^31 rows); a SUM term that fits int32 is added to its
// cell, and when the add wraps the cell past the int32 range (signs of the
// old value and the term agree, the new value's differs) the lost 2^32 goes
// to the global table; a wider term goes to the global table directly.  The
// cell plus the global corrections is the exact 64-bit sum.
__device__ __forceinline__ void table_add(const Table& t, int which, int64_t gid, int64_t v) {
    const int lc = (int)((t.amap >> (4 * which)) & 15u);
    if (t.loff >= 0 && t.c32 && gid < t.lG && lc != 15) {
        uint32_t* cell = (uint32_t*)(ccq_lds + t.loff) + (lc * t.lG + gid);
        if (which == 0) {
            atomicAdd(cell, (uint32_t)v);
        } else if (v == (int64_t)(int32_t)v) {
            const uint32_t add = (uint32_t)(int32_t)v;
            const int32_t o = (int32_t)atomicAdd(cell, add);
            const int32_t n = (int32_t)((uint32_t)o + add);
            if (((o ^ n) & ((int32_t)v ^ n)) < 0)
                atomicAdd((unsigned long long*)&t.g[which * t.G + gid],
                          (unsigned long long)(v > 0 ? (int64_t(1) << 32) : -(int64_t(1) << 32)));
        } else {
            atomicAdd((unsigned long long*)&t.g[which * t.G + gid], (unsigned long long)v);
        }
    } else if (t.loff >= 0 && !t.c32) {
        atomicAdd((unsigned long long*)(ccq_lds + t.loff) + (which * t.G + gid), (unsigned long long)v);
    } else {
        atomicAdd((unsigned long long*)&t.g[which * t.G + gid], (unsigned long long)v);
    }
}


// ------------------------------------------------------------------ fused kernel

struct WaveLds {
    unsigned char* base;
    int32_t* tn;        // [kMaxRle] staged runs of each column in the current tile
    int64_t* tlo;       // [kMaxRle] run index of each column's first staged run
    int64_t* cur;       // [kMaxRle] run index holding the next tile's first row
    int32_t* run_end;   // [run_cap] run end - tile start, capped at 2^30
    int64_t* run_val;   // [run_cap] run value; for a key column that is not summed, its group-id part
                        // (key value times its radix weight, -1 outside the key's domain)
    uint32_t* tog;      // 64-word toggle bitmap per RLE column
    uint32_t* bnd;      // staged paths: 64-word run-boundary bitmap per RLE column
    int32_t* bpre;      // staged paths: exclusive prefix of boundary popcounts per word
    uint32_t* pmw;      // staged paths: the lanes' surviving-row words
    uint32_t* rcl;      // staged row mode: the row clause's RLE rows, one word per lane
};

// first staged-run slot and capacity of RLE column c in a wave slice
__device__ __forceinline__ int32_t stage_base(const DevPlan& P, int c) { return P.rle[c].stage_base; }
__device__ __forceinline__ int32_t stage_cap(const DevPlan& P, int c) { return P.rle[c].stage_cap; }

// bits 0..b of a word
__device__ __forceinline__ uint32_t bits_le(int b) { return 0xFFFFFFFFu >> (31 - b); }

// the lane's rows of [0, L) at or after lo_valid
__device__ __forceinline__ uint32_t lane_window(int32_t L, int32_t lo_valid) {
    const int32_t b = lane_id() * kRowSpan;
    const int32_t lo = lo_valid - b, hi = L - b;
    uint32_t m = 0xFFFFFFFFu;
    if (lo > 0) m = lo >= 32 ? 0u : m << lo;
    if (hi < 32) m &= hi <= 0 ? 0u : ((1u << hi) - 1u);
    return m;
}

// Stage the runs of every RLE column that overlap [t0, *t1) into LDS and
// build the tile's bitmaps in the same pass (tiles start at multiples of 32
// rows; lane l owns rows [32l, 32l + 32)).  The first 64-run batch of every
// column is loaded in one round trip; further batches follow only for
// columns with more runs in the tile.  A column that would exceed its share
// shrinks *t1 to the end of its last staged run, rounded down to 32 rows, so
// all columns cover the (possibly shorter) tile.  Per column, while a batch
// is in registers:
//   - the run's end, value and (key columns) group-id part (key value times
//     its radix weight, -1 outside the key's domain) go to LDS;
//   - a bit marks the row where the next run starts (boundary bitmap; its
//     word prefixes follow with one wavefront scan), so the staged run holding
//     row r is bpre[r / 32] + popcount(bnd[r / 32] & bits <= r % 32);
//   - with predicates, a toggle marks the rows where the outcome changes from
//     one run to the next; the inclusive prefix XOR of the toggles, started
//     from the outcome of the tile's first run, is the column's pass mask
//     (Section 6 alignment restricted to passing runs).
// Returns the lane's rows in the window [w0, ...) that pass every RLE
// predicate; leaves in W.cur the run holding the next tile's first row.
template <int KMAX>
__device__ __forceinline__ uint32_t stage_tile(const DevPlan& P, const WaveLds& W, int64_t t0, int64_t* t1,
                                               int64_t w0) {
    const int lane = lane_id();
    int64_t e0[KMAX], v0[KMAX], lo[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        e0[c] = INT64_MAX;
        v0[c] = 0;
        lo[c] = 0;
        if (c < P.k_rle) {
            const RleCol& rc = P.rle[c];
            lo[c] = W.cur[c];
            const int64_t i = lo[c] + lane;
            if (i < rc.n_runs) {
                e0[c] = gld(rc.ends, i);
                v0[c] = ld_val(rc.vals, rc.vtype, i);
            }
        }
    }
    uint32_t pm = 0xFFFFFFFFu;
    uint32_t any = 0;             // the open OR clause's rows
    uint32_t rcl = 0;             // the row clause's RLE rows
    bool shrunk = false;
    int64_t last_e[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        last_e[c] = 0;
        if (c >= P.k_rle) continue;
        const RleCol& rc = P.rle[c];
        const int32_t off = stage_base(P, c);
        const int32_t cap = stage_cap(P, c);
        uint32_t* B = W.bnd + c * 64;
        uint32_t* T = W.tog;
        const bool haspred = rc.pred != kPredNone;
        uint32_t first = 0;
        bool carry_pass = false;      // the previous batch's last staged run
        int64_t carry_e = INT64_MAX;
        int32_t n = 0;
        int64_t e = e0[c], v = v0[c];
        for (;;) {
            const bool valid = lo[c] + n + lane < rc.n_runs && n + lane < cap;
            const uint64_t last = wave_ballot(valid && e >= *t1);
            const uint64_t vmask = wave_ballot(valid);
            const int cnt = last ? __builtin_ctzll(last) + 1 : __builtin_popcountll(vmask);
            const bool st = lane < cnt;
            const bool pass = st && (!haspred || pred_pass(rc.pred, rc.lo, rc.hi, rc.set, rc.set_len, v));
            const uint64_t pb = wave_ballot(pass);
            if (n == 0) first = (uint32_t)(pb & 1u);
            else if (haspred && lane == 0 && carry_e < *t1 && carry_pass != ((pb & 1u) != 0)) {
                const uint32_t r = (uint32_t)(carry_e - t0);
                atomicOr(&T[r >> 5], 1u << (r & 31));
            }
            if (st) {
                const int64_t rel = e - t0;
                W.run_end[off + n + lane] = (int32_t)(rel < (1 << 30) ? rel : (1 << 30));
                // a key column that is not summed keeps its group-id part instead of its value
                int64_t keep = v;
                if (rc.key_on && rc.sum_slot < 0 && !rc.keep_value) {
                    const int64_t kv = v >> rc.key_shift;
                    keep = (kv >= 0 && kv < rc.key_card) ? kv * rc.key_stride : -1;
                }
                W.run_val[off + n + lane] = keep;
                if (e < *t1) {
                    const uint32_t r = (uint32_t)rel;
                    atomicOr(&B[r >> 5], 1u << (r & 31));
                    // the next run's outcome (within this batch; across batches: below)
                    if (haspred && lane < cnt - 1 && pass != (((pb >> (lane + 1)) & 1u) != 0))
                        atomicOr(&T[r >> 5], 1u << (r & 31));
                }
            }
            carry_pass = ((pb >> (cnt - 1)) & 1u) != 0;
            carry_e = __shfl(e, cnt - 1, 64);
            last_e[c] = carry_e;
            n += cnt;
            if (last) break;
            if (n >= cap) {
                const int64_t cut = t0 + ((last_e[c] - t0) & ~(int64_t)(kRowSpan - 1));
                if (cut < *t1) {
                    *t1 = cut;
                    shrunk = true;
                }
                break;
            }
            const int64_t i = lo[c] + n + lane;
            e = INT64_MAX;
            v = 0;
            if (i < rc.n_runs && n + lane < cap) {
                e = gld(rc.ends, i);
                v = ld_val(rc.vals, rc.vtype, i);
            }
        }
        if (lane == 0) {
            W.tn[c] = n;
            W.tlo[c] = lo[c];
        }
        if (haspred) {
            // the column's pass mask from its toggles (one scratch bitmap, cleared for the next column)
            wave_lds_sync();
            const uint32_t t = T[lane];
            T[lane] = 0;
            uint32_t x = t;
            x ^= x << 1;
            x ^= x << 2;
            x ^= x << 4;
            x ^= x << 8;
            x ^= x << 16;
            const uint64_t par = wave_ballot((__builtin_popcount(t) & 1) != 0);
            const uint32_t flip = ((uint32_t)lanes_below(par) ^ first) & 1u;
            any |= flip ? ~x : x;
            if (!rc.or_next) {
                if (rc.row_clause) rcl = any;
                else pm &= any;
                any = 0;
            }
        }
    }
    wave_lds_sync();
    // boundary prefixes per word
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        if (c >= P.k_rle) continue;
        const int bc = __builtin_popcount(W.bnd[c * 64 + lane]);
        W.bpre[c * 64 + lane] = wave_inclusive_sum_dpp(bc) - bc;
    }
    wave_lds_sync();
    // the run holding row t1: the last staged run unless it ends exactly at t1
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        if (c >= P.k_rle) continue;
        int64_t nxt;
        if (!shrunk) nxt = lo[c] + W.tn[c] - (last_e[c] > *t1 ? 1 : 0);
        else nxt = lo[c] + lds_upper_bound(W.run_end + stage_base(P, c), W.tn[c], (int32_t)(*t1 - t0));
        if (lane == 0) W.cur[c] = nxt;
    }
    if (W.rcl) W.rcl[lane] = rcl;
    wave_lds_sync();
    return pm & lane_window((int32_t)(*t1 - t0), (int32_t)(max(t0, w0) - t0));
}

// Group-id part of the RLE keys from the staged runs' precomputed parts
// (idx[c]: the staged run of column c); false (status raised) if a key is
// outside its domain.
template <int KMAX>
__device__ __forceinline__ bool rle_key_part(const DevPlan& P, const WaveLds& W, const int32_t (&idx)[KMAX],
                                             int64_t* gid, int32_t* status) {
    int64_t g = 0;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        if (c < P.k_rle && P.rle[c].key_on) {
            const RleCol& rc = P.rle[c];
            int64_t part = W.run_val[stage_base(P, c) + idx[c]];   // staged as the part
            if (rc.sum_slot >= 0 || rc.keep_value) {                // staged as the value
                const int64_t kv = part >> rc.key_shift;
                part = (kv >= 0 && kv < rc.key_card) ? kv * rc.key_stride : -1;
            }
            ok = ok && part >= 0;
            g += part;
        }
    }
    if (!ok) raise_status(status, -4);
    *gid = g;
    return ok;
}

// consecutive aligned runs of one group, added in registers
template <int KMAX>
struct RegAcc {
    int64_t gid;
    int64_t cnt;
    int64_t rsum[KMAX];   // SUM of each RLE column
};

template <int KMAX>
__device__ __forceinline__ void regacc_flush(const DevPlan& P, const Table& tb, RegAcc<KMAX>& a) {
    if (a.gid >= 0 && a.cnt > 0) {
        table_add(tb, 0, a.gid, a.cnt);
#pragma unroll
        for (int c = 0; c < KMAX; ++c)
            if (c < P.k_rle && P.rle[c].sum_slot >= 0 && a.rsum[c] != 0)
                table_add(tb, 1 + P.rle[c].sum_slot, a.gid, a.rsum[c]);
    }
    a.gid = -1;
    a.cnt = 0;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) a.rsum[c] = 0;
}

// ---- staged paths: run boundaries as bitmaps
//
// Tiles start at multiples of 32 rows and lane l owns the tile's rows
// [32l, 32l + 32).  Once the runs of a tile are staged, every RLE column gets
// a 64-word bitmap with a bit at each row where a new run starts inside the
// tile, and the exclusive prefix of its popcounts per word: the staged run
// holding row r is then bpre[r / 32] + popcount(bnd[r / 32] & bits <= r % 32),
// with no search.  A column with predicates also gets its pass mask: toggles
// where the outcome changes from one run to the next, prefix XOR, started
// from the outcome of the tile's first run (Section 6 alignment restricted to
// passing runs, as in the fast path).

__device__ __forceinline__ void tile_bitmaps_clear(const DevPlan& P, const WaveLds& W) {
    wave_lds_sync();
    for (int c = 0; c < P.k_rle; ++c) W.bnd[c * 64 + lane_id()] = 0;
    wave_lds_sync();
}

// the staged run of column c holding tile row r
__device__ __forceinline__ int32_t bm_run(const WaveLds& W, int c, int32_t r) {
    return W.bpre[c * 64 + (r >> 5)] + __builtin_popcount(W.bnd[c * 64 + (r >> 5)] & bits_le(r & 31));
}

// Run mode on bitmaps: the lane's word is cut into segments at the run
// boundaries of the key and SUM columns; a segment's surviving rows are
// popcount(mask & segment); COUNT += rows and SUM += value * rows per segment
// (Section 7 aggregating phase), consecutive segments of one group added in
// registers first.
template <int KMAX>
__device__ __forceinline__ void tile_run_bits(const DevPlan& P, const WaveLds& W, int64_t t0, int32_t L, uint32_t pm,
                                              const Table& tb, int32_t* status, RegAcc<KMAX>& acc,
                                              int64_t (&pcur)[kMaxIdx]) {
    const int lane = lane_id();
    uint32_t bw[KMAX];
    int32_t pre[KMAX];
    uint32_t U = 0;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        bw[c] = 0;
        pre[c] = 0;
        if (c >= P.k_rle) continue;
        bw[c] = W.bnd[c * 64 + lane];
        pre[c] = W.bpre[c * 64 + lane];
        if (P.rle[c].key_on || P.rle[c].sum_slot >= 0) U |= bw[c];
    }
    // group segments of the tile: cut at the key columns' boundaries; with a
    // global table their pieces meet in LDS slots first
    uint32_t K = 0;
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
        if (c < P.k_rle && P.rle[c].key_on) K |= bw[c];
    int kpre = 0, ktot = 0;
    const int stride = 2 + P.n_sums;
    if (P.seg_slots) kpre = wave_exclusive_sum(__builtin_popcount(K), &ktot);
    if (pm) {
        int s = 0;
        for (;;) {
            const uint32_t above = U & (0xFFFFFFFEu << s);      // boundaries after row s
            const int e = above ? __builtin_ctz(above) : 32;
            const uint32_t seg = (e >= 32 ? 0xFFFFFFFFu : ((1u << e) - 1u)) & (0xFFFFFFFFu << s);
            const int64_t cnt = __builtin_popcount(pm & seg);
            if (cnt) {
                int32_t idx[KMAX];
                int64_t vals[KMAX];
#pragma unroll
                for (int c = 0; c < KMAX; ++c) {
                    idx[c] = 0;
                    vals[c] = 0;
                    if (c < P.k_rle && (P.rle[c].key_on || P.rle[c].sum_slot >= 0)) {
                        idx[c] = pre[c] + __builtin_popcount(bw[c] & bits_le(s));
                        if (P.rle[c].sum_slot >= 0) vals[c] = W.run_val[stage_base(P, c) + idx[c]];
                    }
                }
                int64_t gid;
                if (rle_key_part<KMAX>(P, W, idx, &gid, status)) {
                    if (P.seg_slots) {
                        const int sid = kpre + __builtin_popcount(K & bits_le(s));
                        if (sid < kSegSlots) {
                            unsigned long long* sl = (unsigned long long*)(W.base + P.off_slots) + sid * stride;
                            sl[0] = (unsigned long long)gid;
                            atomicAdd(&sl[1], (unsigned long long)cnt);
#pragma unroll
                            for (int c = 0; c < KMAX; ++c)
                                if (c < P.k_rle && P.rle[c].sum_slot >= 0)
                                    atomicAdd(&sl[2 + P.rle[c].sum_slot], (unsigned long long)(vals[c] * cnt));
                        } else {
                            table_add(tb, 0, gid, cnt);
#pragma unroll
                            for (int c = 0; c < KMAX; ++c)
                                if (c < P.k_rle && P.rle[c].sum_slot >= 0)
                                    table_add(tb, 1 + P.rle[c].sum_slot, gid, vals[c] * cnt);
                        }
                    } else {
                        if (gid != acc.gid) {
                            regacc_flush<KMAX>(P, tb, acc);
                            acc.gid = gid;
                        }
                        acc.cnt += cnt;
#pragma unroll
                        for (int c = 0; c < KMAX; ++c)
                            if (c < P.k_rle && P.rle[c].sum_slot >= 0) acc.rsum[c] += vals[c] * cnt;
                    }
                }
            }
            if (e >= 32) break;
            s = e;
        }
    }
    if (P.seg_slots) {
        // one table add per group segment of the tile, then clear the slots
        wave_lds_sync();
        unsigned long long* sl = (unsigned long long*)(W.base + P.off_slots);
        const int nseg = min(ktot + 1, kSegSlots);
        for (int i = lane; i < nseg; i += 64) {
            unsigned long long* q = sl + i * stride;
            const int64_t cnt = (int64_t)q[1];
            if (cnt) {
                const int64_t gid = (int64_t)q[0];
                table_add(tb, 0, gid, cnt);
                for (int k = 0; k < P.n_sums; ++k)
                    if (q[2 + k]) table_add(tb, 1 + k, gid, (int64_t)q[2 + k]);
            }
            for (int k = 0; k < stride; ++k) q[k] = 0;
        }
        wave_lds_sync();
    }
    if (P.n_idx > 0) {
        // Index points: the point's row must survive; its runs come from the bitmaps
        W.pmw[lane] = pm;
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < kMaxIdx; ++j) {
            if (j >= P.n_idx) continue;
            const IdxCol& ic = P.idx[j];
            int64_t p0 = pcur[j];
            for (;;) {
                const int64_t i = p0 + lane;
                const bool valid = i < ic.n;
                const int64_t pos = valid ? ld_val(ic.pos, ic.ptype, i) : INT64_MAX;
                const bool in = valid && pos < t0 + L;
                const uint64_t m = wave_ballot(in);
                if (in && ic.sum_slot >= 0) {
                    const int32_t rel = (int32_t)(pos - t0);
                    if ((W.pmw[rel >> 5] >> (rel & 31)) & 1u) {
                        int32_t idx[KMAX];
#pragma unroll
                        for (int c = 0; c < KMAX; ++c) {
                            idx[c] = 0;
                            if (c < P.k_rle && P.rle[c].key_on) idx[c] = bm_run(W, c, rel);
                        }
                        int64_t gid;
                        if (rle_key_part<KMAX>(P, W, idx, &gid, status)) {
                            const int64_t v = ld_val(ic.vals, ic.vtype, i);
                            if (v != 0) table_add(tb, 1 + ic.sum_slot, gid, v);
                        }
                    }
                }
                const int c = __builtin_popcountll(m);
                p0 += c;
                if (c < 64) break;
            }
            pcur[j] = p0;
        }
    }
}

// Predicates on Index columns (Table 2: RLE x Index and Index x Index AND,
// idx_in_rle / idx_in_idx, here on 32-row words).  A column's value is 0 at
// the rows it does not list, so only its points can differ from the outcome
// of 0: those points go into a scratch bitmap, and the column's pass mask is
// that bitmap, or its complement (NOT, Section 5.3) when 0 passes.  The
// tile's points start at pcur (not advanced here).
__device__ __forceinline__ uint32_t idx_pred_mask(const DevPlan& P, const WaveLds& W, int64_t t0, int32_t L,
                                                  const int64_t (&pcur)[kMaxIdx], uint32_t pm) {
    const int lane = lane_id();
#pragma unroll
    for (int j = 0; j < kMaxIdx; ++j) {
        if (j >= P.n_idx) continue;
        const IdxCol& ic = P.idx[j];
        if (ic.pred == kPredNone) continue;
        uint32_t* T = W.tog;
        int64_t p0 = pcur[j];
        for (;;) {
            const int64_t i = p0 + lane;
            const bool valid = i < ic.n;
            const int64_t pos = valid ? ld_val(ic.pos, ic.ptype, i) : INT64_MAX;
            const bool in = valid && pos < t0 + L;
            const uint64_t m = wave_ballot(in);
            if (in) {
                const bool pass = pred_pass(ic.pred, ic.lo, ic.hi, ic.set, ic.set_len, ld_val(ic.vals, ic.vtype, i));
                if (pass != (ic.zero_pass != 0)) {
                    const int32_t rel = (int32_t)(pos - t0);
                    atomicOr(&T[rel >> 5], 1u << (rel & 31));
                }
            }
            const int c = __builtin_popcountll(m);
            p0 += c;
            if (c < 64) break;
        }
        wave_lds_sync();
        const uint32_t x = T[lane];
        T[lane] = 0;
        wave_lds_sync();
        const uint32_t m = ic.zero_pass ? ~x : x;
        if (ic.or_rcl && W.rcl) {
            // an OR clause's Index part: the clause holds where its RLE part
            // (the row clause word) or this mask does; the row test that reads
            // the word afterwards then passes every row
            pm &= W.rcl[lane] | m;
            W.rcl[lane] = 0xFFFFFFFFu;
            wave_lds_sync();
        } else {
            pm &= m;
        }
    }
    return pm;
}

// code table lookup (table at LDS byte offset `off`): uint8 tables use
// 254 / 255 for domain / reject
__device__ __forceinline__ uint32_t lut_get(int32_t off, int32_t u8, uint32_t code) {
    if (u8) {
        const uint32_t e = ccq_lds[off + code];
        return e >= 254u ? e + (0xFFFFu - 255u) : e;
    }
    return ((const uint16_t*)(ccq_lds + off))[code];
}

// bits [j*W, j*W + W) of the lane's packed words (j and W compile-time)
template <int W0>
__device__ __forceinline__ uint32_t extract_code(const uint32_t (&wd)[W0 > 0 ? W0 : 1], int j) {
    const int b = j * W0, q = b >> 5, sh = b & 31;
    const uint32_t mask = W0 == 32 ? 0xFFFFFFFFu : ((1u << W0) - 1u);
    if (sh + W0 <= 32) return (wd[q] >> sh) & mask;
    return __builtin_amdgcn_alignbit(wd[q + 1], wd[q], sh) & mask;
}

// ---- fast row path
//
// One bit-packed column of width W0 (14 or 20); no RLE value per row; at
// most one key, the bit-packed column itself, so a row's group is its slot.
// A lane owns 32 consecutive rows of a tile, i.e. W0 whole words of the
// packed stream (tiles start at multiples of 32 rows), held in registers.
//
// RLE predicates never stage runs: each lane takes one run of a 64-run batch
// read straight from HBM, the predicate is evaluated once per run, and a
// toggle is marked at a run's end when the outcome of the next run differs.
// The inclusive prefix XOR of the toggles over the tile, started from the
// outcome of the run holding the tile's first row, is the column's pass
// mask (Section 6 alignment: the AND over columns of these masks is the
// merge of their run ends restricted to passing runs).  Outcomes and
// toggles of a batch are 64-bit lane masks in scalar registers.
//
// A wave walks its tiles as a software pipeline: while tile i is counted,
// the packed words of tile i+1 (only for lanes with surviving rows), the run
// batches of tile i+2 and the Index points of tile i+1 are in flight.  Batch
// loads address through wave-uniform buffer resources, so their addressing
// is scalar work only.

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Wave-uniform buffer resource over the n bytes at p + off, n clamped to
// [0, cap]; a read past them returns zero without a memory access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uni_rsrc(const void* p, int64_t off, int64_t n, int32_t cap) {
    const uint64_t a = (uint64_t)p + (uint64_t)off;
    const uint32_t alo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t ahi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const int32_t nr = __builtin_amdgcn_readfirstlane(n <= 0 ? 0 : (n >= (int64_t)cap ? cap : (int32_t)n));
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)ahi << 32) | alo), (short)0, nr, 0x00020000);
}

// the lanes [0, rem) of a 64-element batch
__device__ __forceinline__ uint64_t batch_lanes(int64_t rem) {
    return rem >= 64 ? ~0ull : (rem <= 0 ? 0ull : ((1ull << rem) - 1ull));
}

// Element i0 + lane of an array of n elements of 4 or 8 bytes (type 1 / 2),
// as two raw dwords (the second one unused for 4-byte elements); zero past
// the array.
struct Raw64 {
    uint32_t lo, hi;
};

__device__ __forceinline__ Raw64 batch_load(const void* p, int32_t type, int64_t i0, int64_t n) {
    const int64_t sz = type == 1 ? 4 : 8;
    const int64_t rem = n - i0;
    const __amdgpu_buffer_rsrc_t rs = uni_rsrc(p, i0 * sz, (rem > 64 ? 64 : rem) * sz, 512);
    const int32_t off = lane_id() * (int32_t)sz;
    Raw64 r;
    r.lo = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    r.hi = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4, 0, 0);
    return r;
}

__device__ __forceinline__ int64_t raw_val(Raw64 r, int32_t type) {
    return type == 1 ? (int64_t)(int32_t)r.lo : (int64_t)(((uint64_t)r.hi << 32) | r.lo);
}

// A register copy made by a vector instruction: state carried from one tile
// to the next is then never the destination of a load still in flight, which
// would make the compiler wait for every load at each later write of it.
__device__ __forceinline__ uint32_t vcopy(uint32_t x) {
    uint32_t y;
    asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
    return y;
}

// run ends (always int64) of runs i0 + lane
__device__ __forceinline__ int64_t batch_ends_val(u32x2 r) {
    return (int64_t)(((uint64_t)vcopy(r.y) << 32) | vcopy(r.x));
}

__device__ __forceinline__ u32x2 batch_ends(const int64_t* ends, int64_t i0, int64_t n) {
    const int64_t rem = n - i0;
    const __amdgpu_buffer_rsrc_t rs = uni_rsrc(ends, i0 * 8, (rem > 64 ? 64 : rem) * 8, 512);
    return __builtin_amdgcn_raw_buffer_load_b64(rs, lane_id() * 8, 0, 0);
}

// a lane's bit of a wave-uniform mask, as the execution mask
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// The current batch of a column: runs b .. b + 63, one per lane, with the
// outcome of each run as a bit of a 64-bit mask.  The raw next batch is read
// again after every pass over two tiles, at the same point of the pass, and
// used in a later pass when the current batch ends; a tile that ends runs of
// more than two batches (runs shorter than 16 rows on average) reads the
// further ones directly.
template <int KMAX>
struct FastRuns {
    int64_t b[KMAX];       // wave-uniform: the batch's first run
    uint64_t valid[KMAX];  // wave-uniform: lanes holding a run
    uint64_t pb[KMAX];     // wave-uniform: lanes whose run passes the predicate
    int64_t e[KMAX];       // this lane's run end
    u32x2 ne[KMAX];        // raw ends of the next batch
    Raw64 nv[KMAX];        // raw values of the next batch
};

// outcome mask of a batch of runs
__device__ __forceinline__ uint64_t batch_pass(const RleCol& rc, Raw64 v, uint64_t valid) {
    return wave_ballot(pred_pass(rc.pred, rc.lo, rc.hi, rc.set, rc.set_len, raw_val(v, rc.vtype))) & valid;
}

__device__ __forceinline__ int64_t rle_runs(const DevPlan& P, int c) { return c < P.k_rle ? P.rle[c].n_runs : 0; }

// make runs b .. b + 63 of column c the current batch (read here)
template <int KMAX>
__device__ __forceinline__ void fast_runs_start(const DevPlan& P, FastRuns<KMAX>& R, int c, int64_t b) {
    const RleCol& rc = P.rle[c];
    const int64_t n = rle_runs(P, c);
    R.b[c] = b;
    R.valid[c] = batch_lanes(n - b);
    R.e[c] = batch_ends_val(batch_ends(rc.ends, b, n));
    R.pb[c] = batch_pass(rc, batch_load(rc.vals, rc.vtype, b, n), R.valid[c]);
}

// read the next batch of every column (again)
template <int KMAX>
__device__ __forceinline__ void fast_runs_next(const DevPlan& P, FastRuns<KMAX>& R) {
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        const RleCol& rc = P.rle[c];
        const int64_t n = rle_runs(P, c);
        R.ne[c] = batch_ends(rc.ends, R.b[c] + 64, n);
        R.nv[c] = batch_load(rc.vals, rc.vtype, R.b[c] + 64, n);
    }
}

// Toggles at the ends of the runs in m (ends in (t0, t1)): the outcome
// changes there.  Toggles of tile A = [t0, tm) go to words 0..63 of the
// column's bitmap, those of B = [tm, t1) to words 64..127.
__device__ __forceinline__ void run_toggles(uint32_t* tog, int64_t e, uint64_t m, int64_t t0, int64_t tm) {
    if (lane_in(m)) {
        const uint32_t rel = e < tm ? (uint32_t)e - (uint32_t)t0 : (uint32_t)e - (uint32_t)tm + (uint32_t)kRowTile;
        atomicOr(&tog[rel >> 5], 1u << (rel & 31));
    }
}

// outcome changes after runs 0..62 of a batch, and after run 63 given the
// outcome (0 or 1) of the run after it
__device__ __forceinline__ uint64_t batch_changes(uint64_t pb, uint64_t pb_next) {
    return pb ^ (pb >> 1) ^ (pb_next << 63);
}

// The lane's rows that pass every RLE predicate in two consecutive tiles,
// A = [t0, tm) and B = [tm, t1) (B may be empty), with one pass over the
// runs.  Tiles are visited in increasing order; a column's current batch
// holds a run ending after t0 and moves on when its last run ends at or
// before t1.
template <int KMAX>
__device__ __forceinline__ void fast_rle_mask(const DevPlan& P, const WaveLds& W, int64_t t0, int64_t tm, int64_t t1,
                                              FastRuns<KMAX>& R, uint32_t& pm_a, uint32_t& pm_b) {
    const int lane = lane_id();
    uint32_t first = 0;   // bit c: the run holding row t0 passes column c
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        if (c >= P.k_rle) continue;
        const RleCol& rc = P.rle[c];
        const int64_t n = rc.n_runs;
        uint32_t* tog = W.tog + c * 128;
        const uint64_t gt = wave_ballot(R.e[c] > t0) & R.valid[c];   // runs ending after t0
        const uint64_t lt = wave_ballot(R.e[c] < t1) & R.valid[c];   // runs ending before t1
        const uint64_t le = wave_ballot(R.e[c] <= t1) & R.valid[c];
        // the first run ending after t0 holds row t0
        if (gt) first |= (uint32_t)((R.pb[c] >> __builtin_ctzll(gt)) & 1u) << c;
        if ((le >> 63) == 0) {
            run_toggles(tog, R.e[c], gt & lt & batch_changes(R.pb[c], R.pb[c] >> 63), t0, tm);
            continue;
        }
        // the batch ends: the next one (read in an earlier pass) is used here
        // and only here
        uint64_t valid = batch_lanes(n - R.b[c] - 64);
        uint64_t pb = batch_pass(rc, R.nv[c], valid);
        int64_t e = batch_ends_val(R.ne[c]);
        run_toggles(tog, R.e[c], gt & lt & batch_changes(R.pb[c], pb & 1u), t0, tm);
        int64_t b = R.b[c] + 64;
        for (;;) {
            const uint64_t in = wave_ballot(e > t0 && e < t1) & valid;
            if (((wave_ballot(e <= t1) & valid) >> 63) == 0) {
                run_toggles(tog, e, in & batch_changes(pb, pb >> 63), t0, tm);
                break;
            }
            // runs shorter than 16 rows: one more batch inside the tiles
            const uint64_t valid3 = batch_lanes(n - b - 64);
            const int64_t e3 = batch_ends_val(batch_ends(rc.ends, b + 64, n));
            const uint64_t pb3 = batch_pass(rc, batch_load(rc.vals, rc.vtype, b + 64, n), valid3);
            run_toggles(tog, e, in & batch_changes(pb, pb3 & 1u), t0, tm);
            b += 64;
            e = e3;
            pb = pb3;
            valid = valid3;
        }
        R.b[c] = b;
        R.valid[c] = valid;
        R.pb[c] = pb;
        R.e[c] = e;
    }
    wave_lds_sync();
    pm_a = 0xFFFFFFFFu;
    pm_b = 0xFFFFFFFFu;
    uint32_t any_a = 0, any_b = 0;   // the open OR clause's rows
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        if (c >= P.k_rle) continue;
        uint32_t* tog = W.tog + c * 128;
        const uint32_t Ta = tog[lane], Tb = tog[64 + lane];
        tog[lane] = 0;
        tog[64 + lane] = 0;
        uint32_t xa = Ta, xb = Tb;
        xa ^= xa << 1;
        xb ^= xb << 1;
        xa ^= xa << 2;
        xb ^= xb << 2;
        xa ^= xa << 4;
        xb ^= xb << 4;
        xa ^= xa << 8;
        xb ^= xb << 8;
        xa ^= xa << 16;
        xb ^= xb << 16;
        // toggles in the words before this one (B after all of A), plus the
        // starting outcome
        const uint64_t para = wave_ballot((__builtin_popcount(Ta) & 1) != 0);
        const uint64_t parb = wave_ballot((__builtin_popcount(Tb) & 1) != 0);
        const uint32_t fa = ((uint32_t)lanes_below(para) ^ (first >> c)) & 1u;
        const uint32_t fb = ((uint32_t)lanes_below(parb) ^ (uint32_t)__builtin_popcountll(para) ^ (first >> c)) & 1u;
        any_a |= fa ? ~xa : xa;
        any_b |= fb ? ~xb : xb;
        if (!P.rle[c].or_next) {
            pm_a &= any_a;
            pm_b &= any_b;
            any_a = 0;
            any_b = 0;
        }
    }
}

// the lane's rows of tile [t0, t1) inside the window (rows >= w0)
__device__ __forceinline__ uint32_t fast_window_mask(int64_t t0, int64_t t1, int64_t w0) {
    if (t0 >= w0 && t1 - t0 == kRowTile) return 0xFFFFFFFFu;   // a whole tile inside the window
    const int32_t b = lane_id() * kRowSpan;
    const int32_t lo = (int32_t)(max(t0, w0) - t0) - b;   // first valid bit
    const int32_t hi = (int32_t)(t1 - t0) - b;            // one past the last
    uint32_t m = 0xFFFFFFFFu;
    if (lo > 0) m = lo >= 32 ? 0u : m << lo;
    if (hi < 32) m &= hi <= 0 ? 0u : ((1u << hi) - 1u);
    return m;
}

// Count the lane's 32 rows into the lane-replicated LDS table (slot-major,
// 2^rep_shift replicas, uint32): the lanes of a wave never hit the same
// address, whatever the skew of the codes.  Slot G counts rows whose key is
// out of its domain, slot G + 1 rejected rows.  Branch free: each batch of
// kFastBatch rows first does all its code-table reads, then all its table adds.
// W0 <= 14: the uint8 code table sits at LDS offset 0 with the reject entry
// at index 2^W0.  Wider columns test a code range; key = (base + code) >>
// shift.  A SUM of the column is accumulated over codes (uint64, same
// replicas); the flush adds base * count.
constexpr int kFastBatch = 8;

template <int W0, bool SUMBP, bool BIG, bool ONES>
__device__ __forceinline__ void fast_rows(const DevPlan& P, const uint32_t (&wd)[W0], uint32_t pm,
                                          const uint8_t* lut, uint32_t* cnt) {
    const int lane = lane_id();
    const BpCol& bc = P.bp[0];
    const uint32_t G = (uint32_t)P.n_groups;
    const uint32_t rep_sh = (uint32_t)P.fast_rep_shift;
    const uint32_t lane_part = (uint32_t)(lane & ((1 << rep_sh) - 1));
    const uint32_t lane_bytes = lane_part * 4u, sh_bytes = rep_sh + 2u;
    unsigned long long* csum = (unsigned long long*)(ccq_lds + P.fast_sum_off);
    const uint32_t reject = G + 1;
    const int32_t npm = (int32_t)~pm;
#pragma unroll
    for (int h = 0; h < kRowSpan; h += kFastBatch) {
        uint32_t slot[kFastBatch];
        uint32_t code[kFastBatch];
#pragma unroll
        for (int j = 0; j < kFastBatch; ++j) {
            const uint32_t c = extract_code<W0>(wd, h + j);
            const bool keep = (pm >> (h + j)) & 1u;
            code[j] = c;
            if constexpr (W0 <= kLutMaxBits && !BIG && ONES) {
                // removed rows read the all-ones code, whose entry rejects
                const uint32_t all = (uint32_t)__builtin_amdgcn_sbfe(npm, h + j, 1);
                slot[j] = lut[c | (all & ((1u << W0) - 1u))];
            } else if constexpr (W0 <= kLutMaxBits && !BIG) {
                slot[j] = lut[keep ? c : (1u << W0)];
            } else {
                uint32_t s = (c - bc.code_lo < bc.code_span) ? 0u : reject;
                if (bc.key >= 0 && s == 0u) {
                    const int64_t kv = (bc.base + (int64_t)c) >> bc.key_shift;
                    s = (kv >= 0 && kv < bc.key_card) ? (uint32_t)(kv - bc.key_lo) : G;
                }
                slot[j] = keep ? s : reject;
            }
        }
#pragma unroll
        for (int j = 0; j < kFastBatch; ++j) {
            atomicAdd((uint32_t*)((unsigned char*)cnt + ((slot[j] << sh_bytes) + lane_bytes)), 1u);
            if constexpr (SUMBP) {
                if (slot[j] < G) atomicAdd(&csum[(slot[j] << rep_sh) + lane_part], (unsigned long long)code[j]);
            }
        }
    }
}

// the slot of a code (a row's group, G = key out of domain, G + 1 = rejected)
template <int W0, bool BIG>
__device__ __forceinline__ uint32_t fast_slot(const BpCol& bc, uint32_t G, const uint8_t* lut, uint32_t code) {
    if constexpr (W0 <= kLutMaxBits && !BIG) {
        return lut[code];
    } else {
        uint32_t slot = (code - bc.code_lo < bc.code_span) ? 0u : G + 1;
        if (bc.key >= 0 && slot == 0u) {
            const int64_t kv = (bc.base + (int64_t)code) >> bc.key_shift;
            slot = (kv >= 0 && kv < bc.key_card) ? (uint32_t)(kv - bc.key_lo) : G;
        }
        return slot;
    }
}

// Index points of the fast path (at most one Index column), in batches of
// 64 that start at multiples of 64 of the point index: the current batch and
// the next are decoded, and the raw batch after them is read when the current
// one is used up.  The points of a pass over two tiles lie in the current
// batch, or at its end and the start of the next one, where (with at most 64
// points in the pass) each lane holds at most one of them; denser passes
// take a slower batch-by-batch route.  A point whose row survives the RLE
// predicates adds its value to the row's group (the Plain x Index case of
// Section 5.1).  The packed words holding its code are read when its pass is
// masked, for surviving points only, and used in the next pass.
struct PointBatch {
    int64_t pos, val;      // point k + lane (pos INT64_MAX past the column)
};

struct FastPoints {
    int64_t k;             // wave-uniform: first point of the current batch
    PointBatch cur, nxt;   // points k + lane and k + 64 + lane
    Raw64 np, nv;          // raw positions and values of points k + 128 + lane
    // the surviving points of the last pass, added in the next one
    uint64_t d_in;         // wave-uniform: lanes holding one
    int64_t d_val;
    uint32_t d_sh, d_lo, d_hi;   // bit offset of its code in the words lo, hi
};

__device__ __forceinline__ int64_t idx_points(const DevPlan& P) {
    return P.n_idx > 0 && P.idx[0].sum_slot >= 0 ? P.idx[0].n : 0;
}

// decode points k + lane
__device__ __forceinline__ void point_decode(const DevPlan& P, int64_t k, Raw64 p, Raw64 v, PointBatch& B) {
    const IdxCol& ic = P.idx[0];
    const bool ok = k + lane_id() < idx_points(P);
    B.pos = ok ? raw_val(p, ic.ptype) : INT64_MAX;
    B.val = ok ? raw_val(v, ic.vtype) : 0;
}

// make the batch at point k (a multiple of 64) current, read here with the
// next one; issue the reads of the one after
__device__ __forceinline__ void fast_points_start(const DevPlan& P, FastPoints& Q, int64_t k) {
    const IdxCol& ic = P.idx[0];
    const int64_t n = idx_points(P);
    Q.k = k;
    point_decode(P, k, batch_load(ic.pos, ic.ptype, k, n), batch_load(ic.vals, ic.vtype, k, n), Q.cur);
    point_decode(P, k + 64, batch_load(ic.pos, ic.ptype, k + 64, n), batch_load(ic.vals, ic.vtype, k + 64, n), Q.nxt);
    Q.np = batch_load(ic.pos, ic.ptype, k + 128, n);
    Q.nv = batch_load(ic.vals, ic.vtype, k + 128, n);
    Q.d_in = 0;
}

// add a surviving point's value to the group of its code
template <int W0, bool BIG>
__device__ __forceinline__ void fast_point_add(const DevPlan& P, int64_t val, uint32_t code, const uint8_t* lut,
                                               int64_t* table) {
    const uint32_t G = (uint32_t)P.n_groups;
    const uint32_t slot = fast_slot<W0, BIG>(P.bp[0], G, lut, code);
    if (slot < G && val != 0) {
        if constexpr (BIG) {
            // a large table keeps no Index sums in LDS: points are few
            atomicAdd((unsigned long long*)&table[(int64_t)(1 + P.idx[0].sum_slot) * G + slot], (unsigned long long)val);
        } else {
            unsigned long long* isum = (unsigned long long*)(ccq_lds + P.fast_isum_off);
            atomicAdd(&isum[slot], (unsigned long long)val);
        }
    }
}

// the code at bit offset sh of the two packed words lo, hi
template <int W0>
__device__ __forceinline__ uint32_t code_at(uint32_t sh, uint32_t lo, uint32_t hi) {
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) & ((1u << W0) - 1u);
}

// the surviving points of the last pass (their words were read a pass ago)
template <int W0, bool BIG>
__device__ __forceinline__ void fast_points_flush(const DevPlan& P, FastPoints& Q, const uint8_t* lut,
                                                  int64_t* table) {
    const uint32_t code = code_at<W0>(Q.d_sh, Q.d_lo, Q.d_hi);
    if (lane_in(Q.d_in)) fast_point_add<W0, BIG>(P, Q.d_val, code, lut, table);
    Q.d_in = 0;
}

// whether the row at pos survives, from the lane masks of tile A = [a0, a1)
// and B = [a1, ...) (every lane takes part: the masks are read across lanes)
__device__ __forceinline__ bool pass_row_survives(int64_t pos, int64_t a0, int64_t a1, uint32_t pma, uint32_t pmb) {
    const uint32_t ra = (uint32_t)pos - (uint32_t)a0, rb = (uint32_t)pos - (uint32_t)a1;
    const uint32_t oa = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((ra >> 5) << 2), (int)pma);
    const uint32_t ob = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((rb >> 5) << 2), (int)pmb);
    return pos < a1 ? ((oa >> (ra & 31)) & 1u) != 0 : ((ob >> (rb & 31)) & 1u) != 0;
}

// The points of the pass over tile A = [a0, a1) and B = [a1, b1) (masks pma,
// pmb): add those of the last pass, find these, and read the words under the
// surviving ones.
template <int W0, bool BIG>
__device__ __forceinline__ void fast_points_pass(const DevPlan& P, FastPoints& Q, int64_t a0, int64_t a1, int64_t b1,
                                                 uint32_t pma, uint32_t pmb, const uint8_t* lut, int64_t* table) {
    const IdxCol& ic = P.idx[0];
    const BpCol& bc = P.bp[0];
    const int64_t npts = idx_points(P);
    if (npts == 0) return;
    fast_points_flush<W0, BIG>(P, Q, lut, table);
    uint64_t in = wave_ballot(Q.cur.pos >= a0 && Q.cur.pos < b1);
    int64_t pos = Q.cur.pos, val = Q.cur.val;
    if (wave_ballot(Q.cur.pos < b1) >> 63) {
        // the current batch ends inside the pass: the next one becomes current
        const int64_t first = Q.k + __builtin_ctzll(wave_ballot(Q.cur.pos >= a0));
        const uint64_t in2 = wave_ballot(Q.nxt.pos < b1);
        if ((in2 & in) != 0 || (in2 >> 63) != 0) {
            // more than 64 points in the pass: batch by batch with the words
            // read here, then batches again at the first point after the pass
            int64_t g = first;
            for (;;) {
                PointBatch B;
                point_decode(P, g, batch_load(ic.pos, ic.ptype, g, npts), batch_load(ic.vals, ic.vtype, g, npts), B);
                const uint64_t in3 = wave_ballot(B.pos < b1);
                const bool live3 = pass_row_survives(B.pos, a0, a1, pma, pmb) && lane_in(in3);
                const int64_t wq = live3 ? (B.pos * W0) >> 5 : 0;
                uint32_t lo = 0, hi = 0;
                if (live3) {
                    lo = gld(bc.packed, wq);
                    hi = gld(bc.packed, wq + 1);
                }
                if (live3) fast_point_add<W0, BIG>(P, B.val, code_at<W0>((uint32_t)(B.pos * W0) & 31u, lo, hi), lut, table);
                const int32_t k = __builtin_popcountll(in3);
                g += k;
                if (k < 64) break;
            }
            fast_points_start(P, Q, g & ~(int64_t)63);
            return;
        }
        if (lane_in(in2)) {
            pos = Q.nxt.pos;
            val = Q.nxt.val;
        }
        in |= in2;
        Q.k += 64;
        Q.cur = Q.nxt;
        point_decode(P, Q.k + 64, Q.np, Q.nv, Q.nxt);
        Q.np = batch_load(ic.pos, ic.ptype, Q.k + 128, npts);
        Q.nv = batch_load(ic.vals, ic.vtype, Q.k + 128, npts);
    }
    const uint64_t live = wave_ballot(pass_row_survives(pos, a0, a1, pma, pmb)) & in;
    // the words under the surviving points, from the pass's stretch of the stream
    const int64_t tw = (a0 >> 5) * W0;
    const __amdgpu_buffer_rsrc_t rs = uni_rsrc(bc.packed, tw * 4, (bc.n_words - tw) * 4, (128 * W0 + 2) * 4);
    constexpr int32_t kNone = 0x40000000;
    const int32_t off = lane_in(live) ? (int32_t)((((uint32_t)pos - (uint32_t)a0) * (uint32_t)W0) >> 5) * 4 : kNone;
    Q.d_lo = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    Q.d_hi = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4, 0, 0);
    Q.d_in = live;
    Q.d_val = val;
    Q.d_sh = (uint32_t)(pos * W0) & 31u;
}

// The fast path counts rows by lane-words, the 32 rows from a multiple of 32
// that one lane covers.  A lane-word whose rows all fail the RLE predicates
// needs no work; the others are gathered from consecutive tiles into batches
// of 64, one per lane, so the row loop runs only on lane-words with rows that
// can count.  Tiles are masked in order; a batch's packed words are read when
// it is complete and counted once the next batch is complete.
template <int KMAX, int W0>
struct FastState {
    FastRuns<KMAX> R;
    FastPoints Q;
    int64_t w0, w1;
    int64_t t0, t1;        // the next tile to mask ([t0, t0) after the last)
    int64_t lw0;           // the wave's first lane-word
    int64_t left, all;     // tiles still to mask, of all
    uint32_t f_pm, f_lw;   // the batch being gathered (lanes below f_n): mask, lane-word - lw0
    int32_t f_n;
    bool pend;             // the second of two tiles masked together is still to gather
    uint32_t pend_pm;
    int64_t pend_a0;
};

// Issue priority from the share of the wave's tiles still ahead: waves that
// fall behind are picked first, so the waves of a compute unit (whose issue
// order otherwise favours the oldest) finish their equal slices together.
__device__ __forceinline__ void balance_priority(int64_t left, int64_t all) {
    if (left * 2 > all) __builtin_amdgcn_s_setprio(3);
    else if (left * 4 > all) __builtin_amdgcn_s_setprio(2);
    else if (left * 8 > all) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// Mask the next tile, take its points and add its active lane-words to the
// batch being gathered.  Returns true when that completes a batch of 64,
// which is then in (r_pm, r_lw).
template <int KMAX, int W0, bool BIG>
__device__ __forceinline__ bool fast_tile(const DevPlan& P, const WaveLds& W, FastState<KMAX, W0>& S,
                                          uint32_t& r_pm, uint32_t& r_lw, const uint8_t* lut, int64_t* table) {
    const int lane = lane_id();
    uint32_t pm;
    int64_t a0;
    if (S.pend) {
        // the second tile of the last pair
        pm = S.pend_pm;
        a0 = S.pend_a0;
        S.pend = false;
    } else {
        // mask the next two tiles in one pass over the runs
        a0 = S.t0;
        const int64_t a1 = S.t1;
        const int64_t b1 = a1 < S.w1 ? min(((a1 >> kTileShift) + 1) << kTileShift, S.w1) : a1;
        balance_priority(S.left, S.all);
        S.left -= 2;
        uint32_t pmb;
        fast_rle_mask<KMAX>(P, W, a0, a1, b1, S.R, pm, pmb);
        pm &= fast_window_mask(a0, a1, S.w0);
        pmb &= fast_window_mask(a1, b1, S.w0);
        fast_points_pass<W0, BIG>(P, S.Q, a0, a1, b1, pm, pmb, lut, table);
        fast_runs_next<KMAX>(P, S.R);
        if (b1 > a1) {
            S.pend = true;
            S.pend_pm = pmb;
            S.pend_a0 = a1;
        }
        S.t0 = b1;
        S.t1 = b1 < S.w1 ? min(((b1 >> kTileShift) + 1) << kTileShift, S.w1) : b1;
    }
    // the k-th active lane-word goes to lane f_n + k of the batch, wrapping
    // into the next batch past 64; the inactive ones fill the other lanes so
    // the lanes are permuted
    const uint64_t act = wave_ballot(pm != 0);
    const int32_t k = __builtin_popcountll(act);
    const int32_t below = lanes_below(act);
    const int32_t pos = (S.f_n + (pm != 0 ? below : k + lane - below)) & 63;
    const uint32_t lw = (uint32_t)((a0 >> 5) - S.lw0) + (uint32_t)lane;
    const uint32_t v_pm = (uint32_t)__builtin_amdgcn_ds_permute(pos << 2, (int)pm);
    const uint32_t v_lw = (uint32_t)__builtin_amdgcn_ds_permute(pos << 2, (int)lw);
    const bool mine = lane >= S.f_n && lane < S.f_n + k;
    const uint32_t g_pm = mine ? v_pm : S.f_pm;
    const uint32_t g_lw = mine ? v_lw : S.f_lw;
    if (S.f_n + k < 64) {
        S.f_pm = g_pm;
        S.f_lw = g_lw;
        S.f_n += k;
        return false;
    }
    r_pm = g_pm;
    r_lw = g_lw;
    const int32_t rem = S.f_n + k - 64;
    S.f_pm = lane < rem ? v_pm : 0u;
    S.f_lw = lane < rem ? v_lw : 0u;
    S.f_n = rem;
    return true;
}

// The packed words of a batch: lane-word lw0 + lw of each lane with rows
// (pm != 0); the others read nothing.  Lane-words are in increasing order
// over the lanes that have rows.
template <int W0>
__device__ __forceinline__ void batch_words(const BpCol& bc, int64_t lw0, uint32_t lw, uint32_t pm,
                                            uint32_t (&wd)[W0]) {
    constexpr int32_t kNone = 0x40000000;
    const uint64_t act = wave_ballot(pm != 0);
    if (act == 0) {
        for (int i = 0; i < W0; ++i) wd[i] = 0;
        return;
    }
    const uint32_t lw_first = (uint32_t)__builtin_amdgcn_readlane((int)lw, __builtin_ctzll(act));
    const uint32_t lw_last = (uint32_t)__builtin_amdgcn_readlane((int)lw, 63 - __builtin_clzll(act));
    const int64_t first_word = (lw0 + lw_first) * W0;
    const int64_t span = (int64_t)(lw_last - lw_first + 1) * W0;   // words from the first lane-word on
    const int64_t avail = bc.n_words - first_word;
    const int64_t rel = (int64_t)(lw - lw_first) * W0;             // this lane's first word from there
    if (span * 4 <= 0x7FFFFFFFll && avail >= span) {
        const __amdgpu_buffer_rsrc_t rs = uni_rsrc(bc.packed, first_word * 4, span * 4, 0x7FFFFFFF);
        const int32_t off = pm ? (int32_t)rel * 4 : kNone;
#pragma unroll
        for (int i = 0; i < W0 / 2; ++i) {
            const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off + 8 * i, 0, 0);
            wd[2 * i] = v.x;
            wd[2 * i + 1] = v.y;
        }
    } else {
        // a batch spread over more than 2 GB of the stream, or the stream's
        // end inside it: word by word from global memory
#pragma unroll
        for (int i = 0; i < W0; ++i) {
            const int64_t q = first_word + rel + i;
            wd[i] = pm && q < bc.n_words ? gld(bc.packed, q) : 0u;
        }
    }
}

// One wavefront over rows [w0, w1) of the plan's window, fast row path.
template <int KMAX, int W0, bool SUMBP, bool BIG, bool ONES>
__device__ __forceinline__ void wave_range_fast(const DevPlan& P, const WaveLds& W, int64_t w0, int64_t w1,
                                                const uint8_t* lut, uint32_t* cnt, int64_t* table) {
    if (w0 >= w1) return;
    const int lane = lane_id();
    const BpCol& bc = P.bp[0];
    FastState<KMAX, W0> S;
    S.w0 = w0;
    S.w1 = w1;
    S.t0 = w0 & ~(int64_t)31;
    S.t1 = min(((S.t0 >> kTileShift) + 1) << kTileShift, w1);
    S.lw0 = S.t0 >> 5;
    S.all = ((w1 - 1) >> kTileShift) - (S.t0 >> kTileShift) + 1;
    S.left = S.all;
    S.f_pm = 0;
    S.f_lw = 0;
    S.f_n = 0;
    S.pend = false;
    S.pend_pm = 0;
    S.pend_a0 = 0;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        if (c < P.k_rle) {
            W.tog[c * 128 + lane] = 0;
            W.tog[c * 128 + 64 + lane] = 0;
        }
        fast_runs_start(P, S.R, c, c < P.k_rle ? wave_upper_bound(P.rle[c].ends, P.rle[c].n_runs, S.t0) : 0);
    }
    fast_runs_next<KMAX>(P, S.R);
    const int64_t pk = P.n_idx > 0 ? wave_lower_bound_pos(P.idx[0].pos, P.idx[0].ptype, P.idx[0].n, w0) : 0;
    fast_points_start(P, S.Q, pk & ~(int64_t)63);
    wave_lds_sync();
    // batches alternate between two word buffers: a complete batch's words
    // are read, then the batch before it is counted
    uint32_t wa[W0], wb[W0];
    uint32_t pa = 0, pb = 0;
    bool have_b = false;
    for (;;) {
        uint32_t rp = 0, rl = 0;
        bool full = false;
        while ((S.pend || S.t0 < S.t1) && !(full = fast_tile<KMAX, W0, BIG>(P, W, S, rp, rl, lut, table))) {
        }
        if (!full) {
            rp = S.f_pm;
            rl = S.f_lw;
        }
        batch_words<W0>(bc, S.lw0, rl, rp, wa);
        pa = rp;
        if (have_b && wave_ballot(pb != 0)) fast_rows<W0, SUMBP, BIG, ONES>(P, wb, pb, lut, cnt);
        if (!full) {
            if (wave_ballot(pa != 0)) fast_rows<W0, SUMBP, BIG, ONES>(P, wa, pa, lut, cnt);
            break;
        }
        full = false;
        while ((S.pend || S.t0 < S.t1) && !(full = fast_tile<KMAX, W0, BIG>(P, W, S, rp, rl, lut, table))) {
        }
        if (!full) {
            rp = S.f_pm;
            rl = S.f_lw;
        }
        batch_words<W0>(bc, S.lw0, rl, rp, wb);
        pb = rp;
        if (wave_ballot(pa != 0)) fast_rows<W0, SUMBP, BIG, ONES>(P, wa, pa, lut, cnt);
        if (!full) {
            if (wave_ballot(pb != 0)) fast_rows<W0, SUMBP, BIG, ONES>(P, wb, pb, lut, cnt);
            break;
        }
        have_b = true;
    }
    if (idx_points(P) > 0) fast_points_flush<W0, BIG>(P, S.Q, lut, table);
    __builtin_amdgcn_s_setprio(0);
}

// Flush of the fast path's LDS tables into the global group table: add up
// the replicas of each slot; the code-space SUM gets base * count; the
// out-of-domain slot raises the status.
__device__ __forceinline__ void fast_flush(const DevPlan& P, int64_t* table, int32_t* status, bool sum_bp,
                                           const uint32_t* cnt, bool big) {
    const int64_t G = P.n_groups;
    const int R = 1 << P.fast_rep_shift;
    const unsigned long long* csum = (const unsigned long long*)(ccq_lds + P.fast_sum_off);
    const unsigned long long* isum = (const unsigned long long*)(ccq_lds + P.fast_isum_off);
    for (int64_t g = threadIdx.x; g <= G; g += blockDim.x) {
        unsigned long long c = 0, s = 0;
        for (int r = 0; r < R; ++r) {
            c += cnt[g * R + r];
            if (sum_bp && g < G) s += csum[g * R + r];
        }
        if (g == G) {
            if (c) raise_status(status, -4);
            continue;
        }
        if (c) atomicAdd((unsigned long long*)&table[g], c);
        if (sum_bp) {
            const unsigned long long v = s + (unsigned long long)P.bp[0].base * c;
            if (v) atomicAdd((unsigned long long*)&table[(int64_t)(1 + P.bp[0].sum_slot) * G + g], v);
        }
        for (int q = 0; q < (big ? 0 : P.n_idx); ++q) {
            const unsigned long long v = isum[q * G + g];
            if (v && P.idx[q].sum_slot >= 0)
                atomicAdd((unsigned long long*)&table[(int64_t)(1 + P.idx[q].sum_slot) * G + g], v);
        }
    }
}

// ---- generic row path
//
// Row mode when the fast path does not apply: several bit-packed columns of
// any width, RLE values per row (an RLE key or SUM next to a bit-packed
// column), the row clause, Index predicates.  The tile's runs are staged and
// masked by stage_tile; the packed words under lanes with surviving rows are
// staged in LDS.  Lane l then walks its own rows 32l .. 32l + 31, all lanes
// on row j together:
//   - a bit-packed column's code is two staged words funnel-shifted, looked
//     up in the column's code table, which folds its predicates and key slot
//     (a4, the RLE x Plain AND of Section 5.1 per row);
//   - an RLE column's staged run advances by one at each bit of the lane's
//     boundary word, so the run holding the row needs no search (a2);
//   - group id and SUM terms follow (a6); rows of one group that follow each
//     other in a lane add up in registers and reach the table when the group
//     changes (a7), so an RLE key reaches it about once per run.
// Index SUMs are taken per point: each lane takes one of the tile's points
// and, if its row survives, adds the point's value to that row's group.

// consecutive rows of one group in a lane, per SUM slot
struct SlotAcc {
    int64_t gid;          // -1: empty
    int64_t cnt;
    int64_t sum[kMaxAggs];
};

__device__ __forceinline__ void slotacc_init(SlotAcc& a) {
    a.gid = -1;
    a.cnt = 0;
#pragma unroll
    for (int k = 0; k < kMaxAggs; ++k) a.sum[k] = 0;
}

template <bool FULL>
__device__ __forceinline__ void slotacc_flush(const DevPlan& P, const Table& tb, SlotAcc& a) {
    constexpr int NS = FULL ? kMaxAggs : kSmallSums;
    if (a.gid >= 0 && a.cnt > 0) {
        table_add(tb, 0, a.gid, a.cnt);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (k >= P.n_sums || a.sum[k] == 0) continue;
            if (FULL && k < P.n_ext && P.ext[k].kind != kExtSum)     // MIN / MAX: encoded, unsigned maximum
                atomicMax((unsigned long long*)&tb.g[(int64_t)(1 + k) * tb.G + a.gid], (unsigned long long)a.sum[k]);
            else
                table_add(tb, 1 + k, a.gid, a.sum[k]);
        }
    }
    a.gid = -1;
    a.cnt = 0;
#pragma unroll
    for (int k = 0; k < kMaxAggs; ++k) a.sum[k] = 0;
}

// Tile row r (whose lane has staged words): the bit-packed predicates and
// the row clause, the group id from the key columns (ridx: the staged run of
// each RLE column holding r) and the decoded bit-packed values.  False if
// the row fails, or (status raised) if a key is outside its domain.
template <int KMAX, bool FULL>
__device__ __forceinline__ bool row_eval(const DevPlan& P, const WaveLds& W, int32_t r,
                                         const int32_t (&ridx)[KMAX], const int32_t (&luts)[kMaxBp],
                                         int32_t* status, int64_t* gid_out, int64_t (&bpv)[kMaxBp],
                                         const int64_t (&cfirst)[kMaxComp], int64_t (&cv)[kMaxComp]) {
    constexpr int NB = FULL ? kMaxBp : kSmallBp;
    bool pass = true;
    bool dom = false;
    int64_t gid = 0;
    uint32_t codes[kMaxBp];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        bpv[j] = 0;
        codes[j] = 0;
        if (j >= P.n_bp) continue;
        const BpCol& bc = P.bp[j];
        const uint32_t* st = (const uint32_t*)(W.base + bc.stage_off);
        // tiles start at multiples of 32 rows, so the tile's first staged
        // word starts with row 0 and row r sits at bit r * w
        const uint32_t bit = (uint32_t)r * (uint32_t)bc.w;
        const uint32_t q = bit >> 5;
        const uint32_t mask = bc.w == 32 ? 0xFFFFFFFFu : ((1u << bc.w) - 1u);
        const uint32_t code = __builtin_amdgcn_alignbit(st[q + 1], st[q], bit & 31) & mask;
        codes[j] = code;
        bpv[j] = bc.base + (int64_t)code;
        if (luts[j] >= 0) {
            const uint32_t e = lut_get(luts[j], bc.lut_u8, code);
            if (e == kLutReject) pass = false;
            else if (e == kLutDomain) dom = true;
            else if (bc.key >= 0) gid += (int64_t)e * bc.key_stride;
        } else {
            pass = pass && pred_pass(bc.pred, bc.lo, bc.hi, bc.set, bc.set_len, bpv[j]);
            if (bc.key >= 0) {
                const int64_t kv = bpv[j] >> bc.key_shift;
                if (kv < 0 || kv >= bc.key_card) dom = true;
                else gid += (kv - bc.key_lo) * bc.key_stride;
            }
        }
    }
    // composite columns (Section 3.2): a row the Index part lists takes the
    // point's value (the tile's bitmap of listed rows and its word prefixes
    // give the point's index), any other row its base part's; the column's
    // predicate is tested on that value
#pragma unroll
    for (int i = 0; i < kMaxComp; ++i) {
        cv[i] = 0;
        if (!FULL || i >= P.n_comp) continue;
        const CompCol& cc = P.comp[i];
        const uint32_t* lm = (const uint32_t*)(W.base + cc.lds_off);
        const uint32_t w = lm[r >> 5];
        int64_t v = 0;
        if ((w >> (r & 31)) & 1u) {
            const int32_t pre = ((const int32_t*)(lm + 64))[r >> 5];
            v = ld_val(cc.vals, cc.vtype, cfirst[i] + pre + __builtin_popcount(w & ((1u << (r & 31)) - 1u)));
        } else if (cc.rle) {
#pragma unroll
            for (int c = 0; c < KMAX; ++c)
                if (c < P.k_rle && c == cc.src) v = W.run_val[stage_base(P, c) + ridx[c]];
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (b < P.n_bp && b == cc.src) v = bpv[b];
        }
        if (!cc.rle) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (b < P.n_bp && b == cc.src) bpv[b] = v;
        }
        cv[i] = v;
        pass = pass && pred_pass(cc.pred, cc.lo, cc.hi, cc.set, cc.set_len, v);
    }
    if (pass && W.rcl) {
        // the row clause (Section 5.2, RLE mask OR Plain mask): its RLE rows,
        // or a bit-packed part holding on this row's value
        bool in = ((W.rcl[r >> 5] >> (r & 31)) & 1u) != 0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j >= P.n_bp || P.bp[j].or_pred == kPredNone) continue;
            if (P.bp[j].or_bits_words > 0) {
                const uint32_t* ob = (const uint32_t*)(ccq_lds + P.bp[j].or_bits_lds_off);
                in = in || ((ob[codes[j] >> 5] >> (codes[j] & 31)) & 1u) != 0;
            } else {
                in = in || pred_pass(P.bp[j].or_pred, P.bp[j].or_lo, P.bp[j].or_hi, P.bp[j].or_set,
                                     P.bp[j].or_set_len, bpv[j]);
            }
        }
        pass = in;
    }
    if (pass && P.any_rle_row) {
        int64_t g2;
        if (rle_key_part<KMAX>(P, W, ridx, &g2, status)) gid += g2;
        else pass = false;
    }
    if (pass && dom) {
        raise_status(status, -4);
        pass = false;
    }
    *gid_out = gid;
    return pass;
}

// the value of RLE column c at the row: its staged run's, or a composite
// column's point value where its Index part lists the row
template <int KMAX, bool FULL>
__device__ __forceinline__ int64_t rle_row_val(const DevPlan& P, const WaveLds& W, int c,
                                               const int32_t (&ridx)[KMAX], const int64_t (&cv)[kMaxComp]) {
    int64_t v = W.run_val[stage_base(P, c) + ridx[c]];
    if constexpr (FULL) {
#pragma unroll
        for (int i = 0; i < kMaxComp; ++i)
            if (i < P.n_comp && P.comp[i].rle && P.comp[i].src == c) v = cv[i];
    }
    return v;
}

// OR of a word over the wave
__device__ __forceinline__ uint32_t wave_or32(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= (uint32_t)__shfl_xor((int)x, o, 64);
    return x;
}

// The common instance's pass over the lane's 32 rows, in two phases.
// Phase 1 goes column by column, so each column's plan fields are read
// once per tile: a bit-packed column's code decides, for every row of the
// lane, the row's pass bit (a code-table reject or a failed predicate), its
// key slot and its part of the row clause; an RLE key column adds its staged
// run's group-id part (the run holding row r is the lane's first run plus
// the boundaries at rows <= r).  Phase 2 adds the surviving rows to the group
// table, consecutive rows of one group through the register accumulator.
template <int KMAX>
__device__ __forceinline__ void lane_rows_two_phase(const DevPlan& P, const WaveLds& W, uint32_t pm,
                                                    const int32_t (&luts)[kMaxBp], const Table& tb,
                                                    int32_t* status, SlotAcc& acc) {
    const int lane = lane_id();
    uint32_t live = pm;
    uint32_t dom = 0;
    int32_t gid[kRowSpan];
#pragma unroll
    for (int r = 0; r < kRowSpan; ++r) gid[r] = 0;
    const bool rcl = W.rcl != nullptr;
    uint32_t orin = rcl ? W.rcl[lane] : 0u;

    // phase 1, bit-packed columns (tiles start at multiples of 32 rows, so
    // the lane's row s0 = 32 lane sits at bit s0 w of the staged words: word
    // lane w, bit 0)
#pragma unroll
    for (int j = 0; j < kSmallBp; ++j) {
        if (j >= P.n_bp) continue;
        const BpCol& bc = P.bp[j];
        const uint32_t* st = (const uint32_t*)(W.base + bc.stage_off);
        const uint32_t w = (uint32_t)bc.w;
        const uint32_t mask = w == 32 ? 0xFFFFFFFFu : ((1u << w) - 1u);
        const uint32_t q0 = (uint32_t)lane * w;
        const int64_t base = bc.base;
        const bool key = bc.key >= 0;
        const int32_t stride = (int32_t)bc.key_stride;
        const bool or_on = rcl && bc.or_pred != kPredNone;
        const bool or_bits = or_on && bc.or_bits_words > 0;
        const uint32_t* ob = (const uint32_t*)(ccq_lds + bc.or_bits_lds_off);
        const int lut = luts[j];
        if (lut >= 0) {
            const int32_t u8 = bc.lut_u8;
#pragma unroll
            for (int r = 0; r < kRowSpan; ++r) {
                const uint32_t b = (uint32_t)r * w;
                const uint32_t q = q0 + (b >> 5);
                const uint32_t code = __builtin_amdgcn_alignbit(st[q + 1], st[q], b & 31) & mask;
                const uint32_t e = lut_get(lut, u8, code);
                if (e == kLutReject) live &= ~(1u << r);
                else if (e == kLutDomain) dom |= 1u << r;
                else if (key) gid[r] += (int32_t)e * stride;
                if (or_bits) {
                    if ((ob[code >> 5] >> (code & 31)) & 1u) orin |= 1u << r;
                } else if (or_on && pred_pass(bc.or_pred, bc.or_lo, bc.or_hi, bc.or_set, bc.or_set_len,
                                              base + (int64_t)code)) {
                    orin |= 1u << r;
                }
            }
        } else {
            const int32_t pk = bc.pred;
            const int64_t lo = bc.lo, hi = bc.hi;
            const int32_t shift = bc.key_shift;
            const int64_t card = bc.key_card, klo = bc.key_lo;
#pragma unroll
            for (int r = 0; r < kRowSpan; ++r) {
                const uint32_t b = (uint32_t)r * w;
                const uint32_t q = q0 + (b >> 5);
                const uint32_t code = __builtin_amdgcn_alignbit(st[q + 1], st[q], b & 31) & mask;
                const int64_t v = base + (int64_t)code;
                if (!pred_pass(pk, lo, hi, bc.set, bc.set_len, v)) live &= ~(1u << r);
                if (key) {
                    const int64_t kv = v >> shift;
                    if (kv < 0 || kv >= card) dom |= 1u << r;
                    else gid[r] += (int32_t)(kv - klo) * stride;
                }
                if (or_bits) {
                    if ((ob[code >> 5] >> (code & 31)) & 1u) orin |= 1u << r;
                } else if (or_on && pred_pass(bc.or_pred, bc.or_lo, bc.or_hi, bc.or_set, bc.or_set_len, v)) {
                    orin |= 1u << r;
                }
            }
        }
    }

    // phase 1, RLE key columns
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        if (c >= P.k_rle || !P.any_rle_row || !P.rle[c].key_on) continue;
        const RleCol& rc = P.rle[c];
        const uint32_t bw = W.bnd[c * 64 + lane];
        const int32_t i0 = W.bpre[c * 64 + lane];
        const int64_t* rv = W.run_val + stage_base(P, c);
        const bool val = rc.sum_slot >= 0 || rc.keep_value;      // staged as the value, not the part
        const int32_t shift = rc.key_shift;
        const int64_t card = rc.key_card, stride = rc.key_stride;
#pragma unroll
        for (int r = 0; r < kRowSpan; ++r) {
            int64_t part = rv[i0 + __builtin_popcount(bw & bits_le(r))];
            if (val) {
                const int64_t kv = part >> shift;
                part = (kv >= 0 && kv < card) ? kv * stride : -1;
            }
            if (part < 0) dom |= 1u << r;
            else gid[r] += (int32_t)part;
        }
    }
    if (rcl) live &= orin;
    dom &= live;
    if (dom) {
        raise_status(status, -4);
        live &= ~dom;
    }

    // phase 2: the surviving rows into the table
    if (!live) return;
    uint32_t sbw[KMAX];
    int32_t si0[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        sbw[c] = 0;
        si0[c] = 0;
        if (c < P.k_rle && P.rle[c].sum_slot >= 0) {
            sbw[c] = W.bnd[c * 64 + lane];
            si0[c] = W.bpre[c * 64 + lane];
        }
    }
#pragma unroll
    for (int r = 0; r < kRowSpan; ++r) {
        if (!((live >> r) & 1u)) continue;
        const int64_t g = gid[r];
        if (g != acc.gid) {
            slotacc_flush<false>(P, tb, acc);
            acc.gid = g;
        }
        acc.cnt += 1;
#pragma unroll
        for (int k = 0; k < kSmallSums; ++k) {
            if (k >= P.n_sums) continue;
            int64_t term = 0;
#pragma unroll
            for (int c = 0; c < KMAX; ++c)
                if (c < P.k_rle && P.rle[c].sum_slot == k)
                    term = W.run_val[stage_base(P, c) + si0[c] + __builtin_popcount(sbw[c] & bits_le(r))];
#pragma unroll
            for (int b = 0; b < kSmallBp; ++b) {
                if (b < P.n_bp && P.bp[b].sum_slot == k) {
                    const BpCol& bc = P.bp[b];
                    const uint32_t* st = (const uint32_t*)(W.base + bc.stage_off);
                    const uint32_t w = (uint32_t)bc.w;
                    const uint32_t bb = (uint32_t)r * w;
                    const uint32_t q = (uint32_t)lane * w + (bb >> 5);
                    const uint32_t mask = w == 32 ? 0xFFFFFFFFu : ((1u << w) - 1u);
                    term = bc.base + (int64_t)(__builtin_amdgcn_alignbit(st[q + 1], st[q], bb & 31) & mask);
                }
            }
            acc.sum[k] += term;
        }
    }
}

template <int KMAX, bool FULL>
__device__ __forceinline__ void tile_row_generic(const DevPlan& P, const WaveLds& W, int64_t t0, int32_t L,
                                                 uint32_t pm, const Table& tb, int32_t* status,
                                                 int64_t (&pcur)[kMaxIdx], int64_t (&ccur)[kMaxComp],
                                                 const int32_t (&luts)[kMaxBp], SlotAcc& acc) {
    constexpr int NB = FULL ? kMaxBp : kSmallBp;
    constexpr int NS = FULL ? kMaxAggs : kSmallSums;
    const int lane = lane_id();
    const uint32_t any = wave_or32(pm);
    if (P.n_idx > 0) W.pmw[lane] = pm;

    // a4: stage only the packed words read by lanes that have surviving rows
    const uint64_t need_lanes = wave_ballot(pm != 0);
    if (any) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j >= P.n_bp) continue;
            const BpCol& bc = P.bp[j];
            const int64_t wbase = (t0 * (int64_t)bc.w) >> 5;
            const int32_t nwords = (int32_t)((((t0 + L) * (int64_t)bc.w - 1) >> 5) + 2 - wbase);
            const uint32_t magic = ((1u << 20) + (uint32_t)bc.w - 1u) / (uint32_t)bc.w;   // ceil(2^20 / w)
            uint32_t* st = (uint32_t*)(W.base + bc.stage_off);
            for (int q = lane; q < nwords; q += 64) {
                // word q is read by lane floor(q / w) and at most two lanes before it
                const int f = (int)(((uint32_t)q * magic) >> 20);
                const int l0 = f >= 2 ? f - 2 : 0;
                const int l1 = f < 63 ? f : 63;
                const uint64_t lanes = l1 >= l0 ? (((2ull << (l1 - l0)) - 1ull) << l0) : 0ull;
                if (need_lanes & lanes) st[q] = gld(bc.packed, wbase + q);
            }
        }
    }
    // composite columns: the tile's listed rows as a bitmap, one word per
    // lane, and the exclusive prefix of the words' popcounts; the tile's
    // points follow the cursor, which moves past them
    int64_t cfirst[kMaxComp];
#pragma unroll
    for (int i = 0; i < kMaxComp; ++i) {
        cfirst[i] = 0;
        if (!FULL || i >= P.n_comp) continue;
        const CompCol& cc = P.comp[i];
        uint32_t* lm = (uint32_t*)(W.base + cc.lds_off);
        lm[lane] = 0;
        wave_lds_sync();
        int64_t p0 = ccur[i];
        cfirst[i] = p0;
        for (;;) {
            const int64_t k = p0 + lane;
            const bool valid = k < cc.n;
            const int64_t pos = valid ? ld_val(cc.pos, cc.ptype, k) : INT64_MAX;
            const bool in = valid && pos < t0 + L;      // the cursor is at the first point >= t0
            if (in) {
                const int32_t rel = (int32_t)(pos - t0);
                atomicOr(&lm[rel >> 5], 1u << (rel & 31));
            }
            const int c = __builtin_popcountll(wave_ballot(in));
            p0 += c;
            if (c < 64) break;
        }
        ccur[i] = p0;
        wave_lds_sync();
        int tot;
        ((int32_t*)(lm + 64))[lane] = wave_exclusive_sum(__builtin_popcount(lm[lane]), &tot);
    }
    wave_lds_sync();

    // the lane's rows: the common instance column by column, then row by
    // row (lane_rows_two_phase); the full instance row j of every lane together
    if (!FULL && any) lane_rows_two_phase<KMAX>(P, W, pm, luts, tb, status, acc);
    if (FULL && any) {
        int32_t ridx[KMAX];
        uint32_t bw[KMAX];
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            ridx[c] = 0;
            bw[c] = 0;
            if (c < P.k_rle && P.any_rle_row &&
                (P.rle[c].key_on || P.rle[c].sum_slot >= 0 || P.rle[c].keep_value)) {
                bw[c] = W.bnd[c * 64 + lane];
                ridx[c] = W.bpre[c * 64 + lane];
            }
        }
        const int32_t s0 = lane * kRowSpan;
        for (int j = 0; j < kRowSpan; ++j) {
            // the staged run holding row s0 + j: boundaries at rows <= s0 + j
#pragma unroll
            for (int c = 0; c < KMAX; ++c) ridx[c] += (int32_t)((bw[c] >> j) & 1u);
            if (!((any >> j) & 1u)) continue;
            if (!((pm >> j) & 1u)) continue;
            int64_t bpv[kMaxBp];
            int64_t cv[kMaxComp];
            int64_t gid;
            if (!row_eval<KMAX, FULL>(P, W, s0 + j, ridx, luts, status, &gid, bpv, cfirst, cv)) continue;
            if (gid != acc.gid) {
                slotacc_flush<FULL>(P, tb, acc);
                acc.gid = gid;
            }
            acc.cnt += 1;
            // SUM terms by slot (static indices keep the accumulators in registers)
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                if (k >= P.n_sums) continue;
                if (FULL && k < P.n_ext) {
                    // MIN, MAX or an expression: the row's operands, then the fold
                    const ExtAcc& e = P.ext[k];
                    int64_t va = 0, vb = 0;
#pragma unroll
                    for (int c = 0; c < KMAX; ++c) {
                        if (c >= P.k_rle) continue;
                        if (e.a_rle && e.a_src == c) va = rle_row_val<KMAX, FULL>(P, W, c, ridx, cv);
                        if (e.b_rle && e.b_src == c) vb = rle_row_val<KMAX, FULL>(P, W, c, ridx, cv);
                    }
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if (b >= P.n_bp) continue;
                        if (!e.a_rle && e.a_src == b) va = bpv[b];
                        if (!e.b_rle && e.b_src == b) vb = bpv[b];
                    }
                    // wrapping int64 arithmetic (equal to the exact value whenever it fits)
                    const uint64_t ua = (uint64_t)va, ub = (uint64_t)vb;
                    const int64_t x = e.op == kOpAdd ? (int64_t)(ua + ub)
                                      : e.op == kOpSub ? (int64_t)(ua - ub)
                                      : e.op == kOpMul ? (int64_t)(ua * ub) : va;
                    if (e.kind == kExtSum) {
                        acc.sum[k] += x;
                    } else {
                        const uint64_t enc = e.kind == kExtMin ? min_enc(x) : max_enc(x);
                        if (enc > (uint64_t)acc.sum[k]) acc.sum[k] = (int64_t)enc;
                    }
                    continue;
                }
                int64_t term = 0;
#pragma unroll
                for (int c = 0; c < KMAX; ++c)
                    if (c < P.k_rle && P.rle[c].sum_slot == k) term = rle_row_val<KMAX, FULL>(P, W, c, ridx, cv);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    if (b < P.n_bp && P.bp[b].sum_slot == k) term = bpv[b];
                acc.sum[k] += term;
            }
        }
    }

    // a5: Index points of the tile (every column's cursor moves past them);
    // a SUM adds each surviving point's value to its row's group
    if (P.n_idx > 0) {
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < kMaxIdx; ++j) {
            if (j >= P.n_idx) continue;
            const IdxCol& ic = P.idx[j];
            int64_t p0 = pcur[j];
            for (;;) {
                const int64_t i = p0 + lane;
                const bool valid = i < ic.n;
                const int64_t pos = valid ? ld_val(ic.pos, ic.ptype, i) : INT64_MAX;
                const bool in = valid && pos < t0 + L;
                const uint64_t m = wave_ballot(in);
                if (in && ic.sum_slot >= 0) {
                    const int32_t rel = (int32_t)(pos - t0);
                    if ((W.pmw[rel >> 5] >> (rel & 31)) & 1u) {
                        int32_t idx[KMAX];
#pragma unroll
                        for (int c = 0; c < KMAX; ++c) {
                            idx[c] = 0;
                            if (c < P.k_rle && (P.rle[c].key_on || P.rle[c].keep_value)) idx[c] = bm_run(W, c, rel);
                        }
                        int64_t bpv[kMaxBp];
                        int64_t cv[kMaxComp];
                        int64_t gid;
                        if (row_eval<KMAX, FULL>(P, W, rel, idx, luts, status, &gid, bpv, cfirst, cv)) {
                            const int64_t v = ld_val(ic.vals, ic.vtype, i);
                            if (v != 0) table_add(tb, 1 + ic.sum_slot, gid, v);
                        }
                    }
                }
                const int c = __builtin_popcountll(m);
                p0 += c;
                if (c < 64) break;
            }
            pcur[j] = p0;
        }
    }
    wave_lds_sync();
}

// ---- workgroup pieces shared by the single-query and the batched kernels

// Load the plan's code tables and clear its LDS tables (whole workgroup;
// ends with a barrier).  luts[j]: LDS offset of column j's code table or -1.
template <int W0, bool BIG>
__device__ __forceinline__ void wg_setup(const DevPlan& P, uint8_t* s_lut, uint32_t* s_cnt, int32_t (&luts)[kMaxBp],
                                         bool load_tables) {
    if (load_tables) {
        if constexpr (W0 > 0 && W0 <= kLutMaxBits && !BIG) {
            const uint32_t* src = (const uint32_t*)P.bp[0].lut;
            uint32_t* dst = (uint32_t*)s_lut;
            for (int i = threadIdx.x; i < P.bp[0].lut_bytes / 4; i += blockDim.x) dst[i] = gld(src, i);
        }
#pragma unroll
        for (int j = 0; j < kMaxBp; ++j) {
            if (W0 <= 0 && j < P.n_bp && P.bp[j].lut) {
                uint32_t* dst = (uint32_t*)(ccq_lds + P.bp[j].lut_lds_off);
                const uint32_t* src = (const uint32_t*)P.bp[j].lut;
                const int n = P.bp[j].lut_bytes / 4;
                for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = gld(src, i);
            }
            if (W0 <= 0 && j < P.n_bp && P.bp[j].or_bits_words > 0) {
                uint32_t* dst = (uint32_t*)(ccq_lds + P.bp[j].or_bits_lds_off);
                const uint32_t* src = P.bp[j].or_bits;
                for (int i = threadIdx.x; i < P.bp[j].or_bits_words; i += blockDim.x) dst[i] = gld(src, i);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kMaxBp; ++j) luts[j] = (W0 <= 0 && j < P.n_bp && P.bp[j].lut) ? P.bp[j].lut_lds_off : -1;
    if constexpr (W0 > 0) {
        if constexpr (!BIG)
            for (int i = threadIdx.x; i < kFastCntWords; i += blockDim.x) s_cnt[i] = 0;
        uint32_t* z = (uint32_t*)(ccq_lds + P.fast_sum_off);
        for (int i = threadIdx.x; i < P.fast_bytes / 4; i += blockDim.x) z[i] = 0;
    } else if (P.table_lds) {
        // int64 cells, or 32-bit cells (compact table), cleared as 32-bit words
        uint32_t* l = (uint32_t*)(ccq_lds + P.table_lds_off);
        const int64_t n =
            P.table_c32 ? (int64_t)P.table_lds_cols * P.table_lds_groups : (int64_t)(1 + P.n_sums) * P.n_groups * 2;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) l[i] = 0;
    }
    __syncthreads();
}

__device__ __forceinline__ WaveLds wave_lds(const DevPlan& P) {
    const int wave = wave_id();
    WaveLds W;
    W.base = ccq_lds + P.lds_shared_bytes + wave * P.lds_wave_bytes;
    W.tn = (int32_t*)(W.base);            // slice header, 256 bytes (host layout reserves it)
    W.tlo = (int64_t*)(W.base + 64);
    W.cur = (int64_t*)(W.base + 128);
    W.run_end = (int32_t*)(W.base + P.off_run_end);
    W.run_val = (int64_t*)(W.base + P.off_run_val);
    W.tog = (uint32_t*)(W.base + P.off_tog);
    W.bnd = (uint32_t*)(W.base + P.off_bnd);
    W.bpre = (int32_t*)(W.base + P.off_bpre);
    W.pmw = (uint32_t*)(W.base + P.off_pmw);
    W.rcl = P.off_rcl >= 0 ? (uint32_t*)(W.base + P.off_rcl) : nullptr;
    return W;
}

// One wavefront over rows [w0, w1) of the plan's window.
template <int KMAX, int W0, bool BIG>
__device__ __forceinline__ void wave_range(const DevPlan& P, const WaveLds& W, int64_t w0, int64_t w1,
                                           const Table& tb, int32_t* status,
                                           const int32_t (&luts)[kMaxBp], const uint8_t* s_lut, uint32_t* cnt) {
    if (w0 >= w1) return;
    if constexpr (W0 > 0) {
        // a large table takes no SUM of the bit-packed column (host rule)
        const bool sum = !BIG && P.bp[0].sum_slot >= 0;
        constexpr bool LUT = W0 <= kLutMaxBits && !BIG;
        if (LUT && P.bp[0].ones_reject) {
            if (sum) wave_range_fast<KMAX, W0, true, BIG, LUT>(P, W, w0, w1, s_lut, cnt, tb.g);
            else wave_range_fast<KMAX, W0, false, BIG, LUT>(P, W, w0, w1, s_lut, cnt, tb.g);
        } else {
            if (sum) wave_range_fast<KMAX, W0, true, BIG, false>(P, W, w0, w1, s_lut, cnt, tb.g);
            else wave_range_fast<KMAX, W0, false, BIG, false>(P, W, w0, w1, s_lut, cnt, tb.g);
        }
    } else {
        int64_t pcur[kMaxIdx];
        for (int c = 0; c < P.k_rle; ++c) {
            const int64_t x = wave_upper_bound(P.rle[c].ends, P.rle[c].n_runs, w0 & ~(int64_t)31);
            if (lane_id() == 0) W.cur[c] = x;
        }
#pragma unroll
        for (int j = 0; j < kMaxIdx; ++j)
            pcur[j] = j < P.n_idx ? wave_lower_bound_pos(P.idx[j].pos, P.idx[j].ptype, P.idx[j].n, w0) : 0;
        int64_t ccur[kMaxComp];
#pragma unroll
        for (int j = 0; j < kMaxComp; ++j)
            ccur[j] = j < P.n_comp ? wave_lower_bound_pos(P.comp[j].pos, P.comp[j].ptype, P.comp[j].n, w0) : 0;
        wave_lds_sync();
        for (int c = 0; c < P.k_rle; ++c) W.bnd[c * 64 + lane_id()] = 0;
        if (P.off_tog >= 0) W.tog[lane_id()] = 0;
        if (P.seg_slots) {
            unsigned long long* sl = (unsigned long long*)(W.base + P.off_slots);
            for (int i = lane_id(); i < kSegSlots * (2 + P.n_sums); i += 64) sl[i] = 0;
        }
        // tiles start at multiples of 32 rows (lane words); the first one may
        // start before the window, whose rows are then masked out
        // (one loop per mode, so each keeps only its own accumulator live)
        int64_t t0 = w0 & ~(int64_t)31;
        if (P.row_mode) {
            // row mode: the common instance (-2) or the full one (-1)
            if constexpr (W0 != 0) {
                SlotAcc sacc;
                slotacc_init(sacc);
                while (t0 < w1) {
                    int64_t t1 = min(((t0 >> kTileShift) + 1) << kTileShift, w1);
                    uint32_t pm = stage_tile<KMAX>(P, W, t0, &t1, w0);
                    const int32_t L = (int32_t)(t1 - t0);
                    pm = idx_pred_mask(P, W, t0, L, pcur, pm);
                    tile_row_generic<KMAX, (W0 == -1)>(P, W, t0, L, pm, tb, status, pcur, ccur, luts, sacc);
                    tile_bitmaps_clear(P, W);
                    t0 = t1;
                }
                slotacc_flush<(W0 == -1)>(P, tb, sacc);
            }
        } else if constexpr (W0 != -2) {
            // run mode: its own instance (0) or the full one (-1)
            RegAcc<KMAX> acc;
            regacc_init(acc);
            while (t0 < w1) {
                int64_t t1 = min(((t0 >> kTileShift) + 1) << kTileShift, w1);
                uint32_t pm = stage_tile<KMAX>(P, W, t0, &t1, w0);
                const int32_t L = (int32_t)(t1 - t0);
                pm = idx_pred_mask(P, W, t0, L, pcur, pm);
                tile_run_bits<KMAX>(P, W, t0, L, pm, tb, status, acc, pcur);
                tile_bitmaps_clear(P, W);
                t0 = t1;
            }
            regacc_flush<KMAX>(P, tb, acc);
        }
    }
}

// Add the workgroup's LDS tables to the plan's global table (whole
// workgroup; starts with a barrier).
template <int KMAX, int W0, bool BIG>
__device__ __forceinline__ void wg_flush(const DevPlan& P, int64_t* table, int32_t* status, const uint32_t* cnt) {
    __syncthreads();
    if constexpr (W0 > 0) {
        fast_flush(P, table, status, !BIG && P.bp[0].sum_slot >= 0, cnt, BIG);
    } else if (P.table_lds && P.table_c32) {
        // compact cells: counts as uint32, sums as int32 (their wraps already
        // went to the global table)
        const uint32_t* l = (const uint32_t*)(ccq_lds + P.table_lds_off);
        const int64_t lg = P.table_lds_groups;
        for (int w = 0; w <= P.n_sums; ++w) {
            const int lc = (int)((P.table_lds_map >> (4 * w)) & 15u);
            if (lc == 15) continue;
            for (int64_t g = threadIdx.x; g < lg; g += blockDim.x) {
                const uint32_t v = l[lc * lg + g];
                if (v) {
                    const int64_t x = w == 0 ? (int64_t)v : (int64_t)(int32_t)v;
                    atomicAdd((unsigned long long*)&table[(int64_t)w * P.n_groups + g], (unsigned long long)x);
                }
            }
        }
    } else if (P.table_lds) {
        const unsigned long long* l = (const unsigned long long*)(ccq_lds + P.table_lds_off);
        const int64_t n = (int64_t)(1 + P.n_sums) * P.n_groups;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            const unsigned long long v = l[i];
            if (v) atomicAdd((unsigned long long*)&table[i], v);
        }
    }
}

template <int KMAX>
__device__ __forceinline__ void regacc_init(RegAcc<KMAX>& acc) {
    acc.gid = -1;
    acc.cnt = 0;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) acc.rsum[c] = 0;
}

// Waves per SIMD the single-query fast row path is compiled for: its
// software pipeline keeps a tile of words in flight per wave, and five waves
// hide the rest of the HBM latency better than four, even at the price of a
// few spilled registers (measured); the staged paths and the batched kernel,
// whose extra state would spill far more, keep the compiler's choice.
constexpr int kFastWaves(int w0) { return w0 > 0 ? 4 : 1; }

// KMAX: bound on RLE columns (register arrays); W0: 0 = run mode or generic
// row mode, else the width of the single bit-packed column of the fast row
// path; BIG: that path with a large table in dynamic LDS.
// One query: every wavefront takes a contiguous slice of whole nominal tiles.
template <int KMAX, int W0, bool BIG>
__global__ __launch_bounds__(kThreads, kFastWaves(W0)) void k_fused(const DevPlan* __restrict__ Pg, int64_t* __restrict__ table,
                                                     int32_t* __restrict__ status, int64_t n_waves_total) {
    const DevPlan& P = *Pg;
    // fast row path: code table and lane-replicated counts in static LDS, so
    // their addresses fold into the ds_* offsets
    __shared__ uint8_t s_lut[(W0 > 0 && W0 <= kLutMaxBits && !BIG) ? (1 << W0) + 16 : 16];
    __shared__ uint32_t s_cnt[(W0 > 0 && !BIG) ? kFastCntWords : 4];
    uint32_t* cnt = BIG ? (uint32_t*)(ccq_lds + P.fast_sum_off) : s_cnt;
    int32_t luts[kMaxBp];
    wg_setup<W0, BIG>(P, s_lut, s_cnt, luts, true);
    Table tb;
    tb.g = table;
    tb.G = P.n_groups;
    tb.loff = (W0 <= 0 && P.table_lds) ? P.table_lds_off : -1;
    tb.c32 = P.table_c32;
    tb.lG = P.table_lds_groups;
    tb.amap = P.table_lds_map;

    const int64_t gw = (int64_t)blockIdx.x * kWaves + wave_id();
    const int64_t tiles_per_wave = (P.n_tiles + n_waves_total - 1) / n_waves_total;
    const int64_t first_tile = P.row_begin >> kTileShift;
    const int64_t w0 = max(P.row_begin, (first_tile + gw * tiles_per_wave) << kTileShift);
    const int64_t w1 = min(P.row_end, (first_tile + (gw + 1) * tiles_per_wave) << kTileShift);

    const WaveLds W = wave_lds(P);
    wave_range<KMAX, W0, BIG>(P, W, w0, w1, tb, status, luts, s_lut, cnt);
    wg_flush<KMAX, W0, BIG>(P, table, status, cnt);
}

// Many queries: workgroups take work items (a query and a range of its
// nominal tiles) from a device counter, split the item's tiles across their
// wavefronts, and add into that query's own table.  Code tables are reloaded
// only when the query changes.
// The batched generic row path (W0 = -2) is compiled for three waves per
// SIMD (168 VGPRs, a few spilled): measured faster on the mixed batch than
// the compiler's 228 VGPRs at two waves.
template <int KMAX, int W0, bool BIG>
__global__ __launch_bounds__(kThreads, W0 == -2 ? 3 : 1) void k_batch(const BatchDev* __restrict__ B, int32_t group,
                                                     unsigned char* __restrict__ ws) {
    __shared__ uint8_t s_lut[(W0 > 0 && W0 <= kLutMaxBits && !BIG) ? (1 << W0) + 16 : 16];
    __shared__ uint32_t s_cnt[(W0 > 0 && !BIG) ? kFastCntWords : 4];
    __shared__ int32_t s_item;
    const BatchGroup& grp = B->groups[group];
    int32_t* counter = B->counters + group;
    int32_t loaded = -1;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= grp.n_items) break;
        const BatchItem it = grp.items[item];
        // The plans do not change during a launch.  Reading a plan through a
        // wave-uniform pointer in the constant address space lets its fields
        // load into scalar registers, as the single-query kernel's plan
        // argument does; through a plain pointer every field would be a flat
        // load into vector registers (and would count against the LDS wait
        // counter as well).
        const uint64_t pbits = (uint64_t)(uintptr_t)B->plans[it.query];
        const uint64_t ubits = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(pbits >> 32)) << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)pbits);
        const DevPlan& P = *(const DevPlan*)(const __attribute__((address_space(4))) DevPlan*)(uintptr_t)ubits;
        int32_t* status = (int32_t*)(ws + B->region[it.query]);
        int64_t* table = (int64_t*)(ws + B->region[it.query] + 256);
        int32_t luts[kMaxBp];
        uint32_t* cnt = BIG ? (uint32_t*)(ccq_lds + P.fast_sum_off) : s_cnt;
        wg_setup<W0, BIG>(P, s_lut, s_cnt, luts, it.query != loaded);
        loaded = it.query;
        Table tb;
        tb.g = table;
        tb.G = P.n_groups;
        tb.loff = (W0 <= 0 && P.table_lds) ? P.table_lds_off : -1;
        tb.c32 = P.table_c32;
        tb.lG = P.table_lds_groups;
        tb.amap = P.table_lds_map;

        // this wave's share of the item's tiles
        const int wave = wave_id();
        const int64_t per = (it.n_tiles + kWaves - 1) / kWaves;
        const int64_t first_tile = P.row_begin >> kTileShift;
        const int64_t a = first_tile + it.first_tile + wave * per;
        const int64_t b = first_tile + it.first_tile + min((int64_t)it.n_tiles, (wave + 1) * per);
        const int64_t w0 = max(P.row_begin, a << kTileShift);
        const int64_t w1 = min(P.row_end, b << kTileShift);

        const WaveLds W = wave_lds(P);
        wave_range<KMAX, W0, BIG>(P, W, w0, w1, tb, status, luts, s_lut, cnt);
        wg_flush<KMAX, W0, BIG>(P, table, status, cnt);
    }
}

}  // namespace ccq
